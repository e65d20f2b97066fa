"""The library gives the same bits whatever the launch mode.

Every kernel of a step is ordered on the handle's stream, and no result depends
on when the host issues the launches.  A run of the half aneurysm (pulsatile
inlet, 200 steps, FP32 and FP16 storage; raw state, observables and FP64 totals
hashed together, tests/launch_digest.py) must give one digest:
  * asynchronously: all steps in one call, one synchronisation;
  * with a synchronisation after every step;
  * on a stream other than the default one;
  * in a child process in which the HIP runtime serialises every kernel launch
    and every copy (AMD_SERIALIZE_KERNEL=3, AMD_SERIALIZE_COPY=3).
"""

import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")

import launch_digest  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
STEPS = 200


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def reference():
    _gpu()
    return {st: launch_digest.digest(st, STEPS, "async") for st in ("f32", "f16")}


@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("mode", ["sync", "stream"])
def test_in_process_modes_agree(reference, storage, mode):
    assert launch_digest.digest(storage, STEPS, mode) == reference[storage]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_serialised_launches_agree(reference, storage):
    env = dict(os.environ, AMD_SERIALIZE_KERNEL="3", AMD_SERIALIZE_COPY="3")
    print(f"child process with serialised launches: {storage}, {STEPS} steps", flush=True)
    out = subprocess.run([sys.executable, os.path.join(HERE, "launch_digest.py"), storage,
                          str(STEPS)], env=env, capture_output=True, text=True, timeout=540)
    assert out.returncode == 0, out.stderr[-2000:]
    line = [x for x in out.stdout.splitlines() if x.startswith("{")][-1]
    assert json.loads(line)["digest"] == reference[storage]
