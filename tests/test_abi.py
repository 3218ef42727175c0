"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/btd.h declares, validates arguments before touching the
device, and its partition / recursion rules agree with the oracle's
independent implementation."""
import ctypes
import os
import re

import pytest

import oracle
from paper_1505_06864_amd import btd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "btd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(btd_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = btd.lib()
    declared = header_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(btd.EXPORTS) == declared


def test_status_strings():
    L = btd.lib()
    for code in (0, 1, 2, 3, -1):
        assert L.btd_status_string(code)


@pytest.mark.parametrize("N,P,depth", [(1, 1, 0), (64, 4, 0), (2048, 512, 1), (4096, 64, 2)])
def test_workspace_bytes_positive(N, P, depth):
    f, s = btd.workspace_bytes(N, 16, P, depth, max_nrhs=4)
    assert f > 0 and s > 0 and f % 256 == 0


@pytest.mark.parametrize("kw", [dict(N=0, M=4), dict(N=8, M=0), dict(N=8, M=btd.BTD_MAX_M + 1),
                                dict(N=8, M=4, P=5), dict(N=8, M=4, P=0), dict(N=8, M=4, depth=-1),
                                dict(N=8, M=4, max_nrhs=0), dict(N=8, M=4, P=3, seps=[0, 4]),
                                dict(N=8, M=4, P=3, seps=[3, 4]), dict(N=8, M=4, P=3, seps=[3, 7]),
                                dict(N=8, M=4, P=3, seps=[5, 3])])
def test_invalid_descriptions_rejected(kw):
    with pytest.raises(btd.BtdError):
        btd.workspace_bytes(**kw)


def test_factor_rejects_bad_arguments_before_device_work():
    L = btd.lib()
    d, _k = btd.make_desc(8, 4, 2, 0, 1)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(256)  # never dereferenced: every call below fails its host checks
    assert L.btd_factor(None, fake, fake, fake, fake, 1 << 20, None, ctypes.byref(h)) == -1
    assert L.btd_factor(ctypes.byref(d), None, fake, fake, fake, 1 << 20, None, ctypes.byref(h)) == -2
    assert L.btd_factor(ctypes.byref(d), fake, None, fake, fake, 1 << 20, None, ctypes.byref(h)) == -3
    assert L.btd_factor(ctypes.byref(d), fake, fake, None, fake, 1 << 20, None, ctypes.byref(h)) == -4
    assert L.btd_factor(ctypes.byref(d), fake, fake, fake, None, 1 << 20, None, ctypes.byref(h)) == -5
    assert L.btd_factor(ctypes.byref(d), fake, fake, fake, ctypes.c_void_p(258), 1 << 20, None,
                        ctypes.byref(h)) == -5
    assert L.btd_factor(ctypes.byref(d), fake, fake, fake, fake, 16, None, ctypes.byref(h)) == -6
    assert L.btd_factor(ctypes.byref(d), fake, fake, fake, fake, 1 << 20, None, None) == -8
    assert L.btd_solve(None, 1, fake, fake, fake, 1 << 20, None) == -1
    fs = L.btd_factor_solve
    assert fs(None, fake, fake, fake, fake, 1 << 20, 1, fake, fake, fake, 1 << 20, None, ctypes.byref(h)) == -1
    assert fs(ctypes.byref(d), fake, fake, fake, fake, 1 << 20, 0, fake, fake, fake, 1 << 20, None,
              ctypes.byref(h)) == -7
    assert fs(ctypes.byref(d), fake, fake, fake, fake, 1 << 20, 2, fake, fake, fake, 1 << 20, None,
              ctypes.byref(h)) == -7
    assert fs(ctypes.byref(d), fake, fake, fake, fake, 1 << 20, 1, None, fake, fake, 1 << 20, None,
              ctypes.byref(h)) == -9
    assert fs(ctypes.byref(d), fake, fake, fake, fake, 1 << 20, 1, fake, None, fake, 1 << 20, None,
              ctypes.byref(h)) == -10
    assert fs(ctypes.byref(d), None, fake, fake, fake, 1 << 20, 1, fake, fake, fake, 1 << 20, None,
              ctypes.byref(h)) == -2
    assert fs(ctypes.byref(d), fake, fake, fake, fake, 16, 1, fake, fake, fake, 1 << 20, None,
              ctypes.byref(h)) == -6
    assert fs(ctypes.byref(d), fake, fake, fake, fake, 1 << 20, 1, fake, fake, fake, 1 << 20, None, None) == -8
    assert L.btd_solve_batch(-1, None, None, None, None, None, 0, None) == -1
    assert L.btd_solve_batch(0, None, None, None, None, None, 0, None) == 0
    assert L.btd_residual(0, 4, 1, fake, fake, fake, fake, fake, fake, fake, None) == -1
    assert L.btd_residual(4, 4, 1, fake, fake, fake, fake, fake, None, fake, None) == -9


def test_partition_matches_oracle():
    for N in range(1, 80):
        for P in range(1, (N + 1) // 2 + 1):
            assert btd.default_separators(N, P) == oracle.partition(N, P), (N, P)
    for N, P in ((2048, 8), (2048, 512), (4096, 64), (4096, 241)):
        assert btd.default_separators(N, P) == oracle.partition(N, P)


def test_balanced_partition_matches_oracle():
    for N in range(1, 70):
        for P in range(1, (N + 1) // 2 + 1):
            for a, b in ((7 / 4, 7 / 6), (1.0, 1.0), (2.5, 1.25), (9.0, 1.0)):
                assert btd.balanced_separators(N, P, a, b) == oracle.balanced_partition(N, P, a, b), (N, P, a, b)
    for N, P in ((3071, 16), (4096, 256), (2048, 512)):
        assert btd.balanced_separators(N, P) == oracle.balanced_partition(N, P)
    for bad in ((6, 4, 1.75, 1.2), (10, 2, 0.5, 1.0), (10, 2, 1.0, 100.0), (0, 1, 1.0, 1.0)):
        with pytest.raises(btd.BtdError):
            btd.balanced_separators(*bad)


def test_coupling_parts_match_oracle():
    for P in range(1, 700):
        for M, R in ((16, 1), (128, 4), (256, 64)):
            assert btd.default_coupling_parts(P, M, R) == oracle.default_m(P, M, R), (P, M, R)


def test_coupling_rows_rule():
    """coupling_rows = k splits a coupling system of P-1 rows into
    floor(P/(k+1)) subsystems (at least 2, Thomas algorithm below 3 rows);
    0 is Eq. SuppMatrM; negative values are rejected before any device work."""
    for P in range(1, 300):
        assert btd.coupling_parts(P, 64, 1, 0) == btd.default_coupling_parts(P, 64, 1)
        for k in (1, 2, 3, 7):
            m = btd.coupling_parts(P, 64, 1, k)
            if P - 1 < 3:
                assert m == 1
            else:
                assert m == max(2, P // (k + 1))
                # every subsystem of the coupling system keeps at least one row
                assert 2 * m - 1 <= P - 1
    with pytest.raises(btd.BtdError):
        btd.coupling_parts(8, 4, 1, -1)
    with pytest.raises(btd.BtdError):
        btd.workspace_bytes(64, 4, 8, 2, 1, None, -1)


@pytest.mark.parametrize("N,M,R,P,depth,seps", [(64, 16, 1, 4, 0, None), (64, 16, 3, 16, 1, None),
                                                (40, 8, 2, 5, 0, [1, 15, 21, 33]), (300, 4, 2, 40, 2, None),
                                                (57, 2, 1, 1, 0, None)])
def test_flop_model_matches_oracle_counter(N, M, R, P, depth, seps):
    """The benchmark's algorithmic FLOP model (LU convention) equals the
    oracle's executed block-operation count converted to the same convention:
    2/3 M^3 per inversion-as-LU, 2 M^3 per block product (including each
    application of an inverse), 2 M^2 R per block x RHS product."""
    from paper_1505_06864_amd import flops, inputs
    A, B, C, F = inputs.diag_dominant(N, M, R, seed=7)
    cnt = oracle.Counter()
    oracle.dm_solve(A, B, C, F, P, seps=seps, depth=depth, counter=cnt)
    fac, sol = flops.totals(N, M, R, P, depth, seps=seps)
    want = 2.0 / 3.0 * M**3 * cnt.inv + 2.0 * M**3 * cnt.mm + 2.0 * M**2 * R * cnt.mr
    assert abs((fac + sol) - want) <= 1e-9 * want


def test_flop_model_large_workload():
    """853.2 GFLOP factor and 2.65 GFLOP solve at N=4096, M=256, R=1, P=64
    (depth 0); the plain Thomas algorithm (P=1) needs 320.6 + 1.61 GFLOP."""
    from paper_1505_06864_amd import flops
    fac, sol = flops.totals(4096, 256, 1, 64, 0)
    assert abs(fac / 1e9 - 853.2) < 0.1 and abs(sol / 1e9 - 2.65) < 0.01
    fac, sol = flops.totals(4096, 256, 1, 1, 0)
    assert abs(fac / 1e9 - 320.6) < 0.1 and abs(sol / 1e9 - 1.61) < 0.01
