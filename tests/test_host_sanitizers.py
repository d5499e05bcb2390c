"""The host lattice builder (csrc/host_lattice.cpp) under AddressSanitizer
and UndefinedBehaviorSanitizer: a g++ build of the builder and the driver
tests/native/host_lattice_check.cpp, fed every compiled lattice card and
user-supplied velocity sets, must finish without a sanitizer report and
agree with the oracle's weights and norms; malformed descriptors are
refused.  CPU only (g++, no GPU code)."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import lattice as OL
from paper_2512_16230_amd import _mrtlb as H
from paper_2512_16230_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CARDS = [W.Q25_RECT, W.Q13_SQUARE, W.Q53_RECT, W.Q33_CUBIC, W.Q21_RECT, W.Q21K_RECT, W.Q45_RECT, W.Q9_RECT,
         W.Q27_RECT] + W.Q17_CASES


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "host_lattice_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "native", "host_lattice_check.cpp"),
           os.path.join(ROOT, "paper_2512_16230_amd", "csrc", "host_lattice.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return out


def _line(card):
    kind = H.KINDS[card.kind]
    free = list(card.free) + [0.0] * (4 - len(card.free))
    c = list(card.c) + [1.0] * (3 - len(card.c))
    return "%d %d 0 %r %r %r %r %d %r %r %r %r" % ((kind, card.d) + tuple(c) + (card.cs2, len(card.free)) + tuple(free))


def _custom_line(card):
    lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
    perm = np.random.default_rng(3).permutation(lat.b)
    c = list(card.c) + [1.0] * (3 - len(card.c))
    head = "%d %d %d %r %r %r %r 0 0 0 0 0" % ((H.KINDS["custom"], lat.d, lat.b) + tuple(c) + (card.cs2,))
    return head + " " + " ".join(str(int(v)) for v in lat.e[perm].ravel()) + " " + \
        " ".join(repr(float(v)) for v in lat.w[perm])


def test_builder_runs_clean_under_sanitizers(driver):
    custom = (W.Q25_RECT, W.Q53_RECT, W.Q13_SQUARE)
    lines = [_line(c) for c in CARDS] + [_custom_line(c) for c in custom]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=300,
                         env=env)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-3000:]
    out = res.stdout.strip().splitlines()
    assert len(out) == len(lines) + 4
    cards = CARDS + list(custom)
    for card, row, custom in zip(cards, out, [False] * len(CARDS) + [True] * 3):
        tok = row.split()
        assert tok[0] == "ok", (card.kind, row)
        B, nlow, worst = int(tok[1]), int(tok[2]), float(tok[3])
        assert worst < 1e-12, card.kind
        w = np.array([float(v) for v in tok[4:4 + B]])
        lat = OL.make_lattice(card.kind, card.c, card.cs2, card.free)
        want = lat.w[np.random.default_rng(3).permutation(lat.b)] if custom else lat.w
        assert np.abs(w - want).max() < 1e-13, card.kind
        assert len(tok) == 4 + B + nlow
    for row in out[len(lines):]:
        assert row.startswith("err %d " % H.MRTLB_EINVAL), row
