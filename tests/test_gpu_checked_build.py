"""The index-checked build (librmrt_checked.so): the FP64 cases of
tests/checked_cases.py, which take every neighbour-index path of the kernels
(odd AA and AB streaming, walls, solid masks, link words, velocity-gradient
initialisation, swapped-layout reads of the companion kernels, persistent,
XCD-ordered and XCD-chunked tile orders, ragged batches with domain groups,
the C = 0 history and the central, Hermite and BHLL collisions), find no
index out of range and give the production library's results (bitwise for every
single-domain case; within rounding where the inserted checks change which
multiply-adds the compiler fuses); with the checks' bound lowered below the
node count, they count the nodes above it."""
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2206_00366_amd")


def _run(lib, out):
    env = dict(os.environ, RMRT_LIBRARY=lib)
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "checked_cases.py"), out],
                         env=env, capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-3000:]
    print(res.stdout, flush=True)
    return res.stdout.splitlines()


def test_checked_build_finds_no_index_out_of_range_and_matches(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    checked = os.path.join(PKG, "librmrt_checked.so")
    assert os.path.exists(checked), "librmrt_checked.so is not built"
    prod_out, chk_out = str(tmp_path / "prod.npz"), str(tmp_path / "checked.npz")
    prod = _run(os.path.join(PKG, "librmrt.so"), prod_out)
    chk = _run(checked, chk_out)
    prod_cases = [ln.split() for ln in prod if ln.startswith("case ")]
    chk_cases = [ln.split() for ln in chk if ln.startswith("case ")]
    assert [c[1] for c in prod_cases] == [c[1] for c in chk_cases] and len(chk_cases) == 13
    assert all(c[2] == "-1" for c in prod_cases)          # the production build has no checks
    assert all(c[2] == "0" for c in chk_cases), chk_cases  # no neighbour index out of range
    a, b = np.load(prod_out), np.load(chk_out)
    assert sorted(a.files) == sorted(b.files)
    exact = 0
    for k in a.files:
        if np.array_equal(a[k], b[k]):
            exact += 1
            continue
        # the inserted checks may change which multiply-adds the compiler
        # fuses (observed: one ulp in the batch after a swapped-layout
        # initialisation); anything beyond rounding is a failure
        fin = np.isfinite(a[k])
        assert np.array_equal(fin, np.isfinite(b[k])), k
        scale = np.abs(a[k][fin]).max()
        assert np.abs(a[k][fin] - b[k][fin]).max() <= 1e-14 * scale, k
    print(f"{exact} of {len(a.files)} outputs bitwise equal", flush=True)
    assert exact >= len(a.files) - 4
    selftest = [ln.split() for ln in chk if ln.startswith("selftest ")]
    assert len(selftest) == 1
    clean, lowered = int(selftest[0][1]), int(selftest[0][2])
    assert clean == 0 and lowered > 0
