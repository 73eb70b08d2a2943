"""The checked build of the library (device-side bounds checks).

Every kernel of libmk_checked.so compares the end of each range of a buffer
it addresses with the end of the allocation behind the pointer it was given
and records a failure for mk_device_checks().  The solves of
tests/device_checks_run.py (run in a child process that loads the checked
build) touch every kernel family: the streaming and matrix-core
contractions in all their forms, the per-trace kernels in every mode, the
series tail and its network, the restart, the stopping rule, the auxiliary
fields, the image, a state round trip and streamed R.  None may report a
range past its allocation.  A second run reports every extent 64 bytes short
(MK_CHECK_SHRINK, a hook of the checked build): the accesses stay where they
are, in bounds, and the checks must fire."""

import os
import subprocess
import sys

import pytest

from gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
RUN = os.path.join(HERE, "device_checks_run.py")


def _run(extra_env, args=()):
    mk = require_gpu()
    if not os.path.exists(mk.CHECKED_LIB_PATH):
        pytest.skip("libmk_checked.so is not built (python -m paper_2106_04649_amd.build --device-checks)")
    env = dict(os.environ, MK_LIBRARY=mk.CHECKED_LIB_PATH, **extra_env)
    say(f"checked build run {args} {extra_env}")
    res = subprocess.run([sys.executable, "-u", RUN, *args], env=env, capture_output=True, text=True, timeout=300)
    say(res.stdout[-4000:])
    assert res.returncode == 0, res.stderr[-4000:]
    return [line for line in res.stdout.splitlines() if line.startswith("case ")]


def test_checked_build_finds_every_range_in_bounds():
    lines = _run({})
    assert len(lines) == 11, lines
    for line in lines:
        assert line.endswith(" checks 0"), line


def test_checks_fire_on_short_extents():
    lines = _run({"MK_CHECK_SHRINK": "64"}, ("--one",))
    assert len(lines) == 1 and not lines[0].endswith(" checks 0"), lines
