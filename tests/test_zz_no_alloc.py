"""hsbuild_forward_static (the entry point that allocates nothing) against
hsbuild_forward with a caller workspace, through the C-ABI.

Two calls in a row on one handle, the second with a smaller basis, so the
second runs in a scratch that still holds the first call's data: each must
equal hsbuild_forward's result bitwise (same kernels, same inputs) and the
oracle to the FP64 bar (relative Frobenius error <= 1e-12; the int8 slice
and the residue forms to <= 1e-10), with the strict lower triangle untouched.
The residue forms take more workspace per basis function, so they run at
bases that fit the scratch.  A problem larger than the static scratch is
refused before anything is enqueued.
"""
import ctypes

import numpy as np
import pytest
import torch

from flapw_cells import make_case
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 3: 1e-10, 4: 1e-10, 5: 1e-10}  # HSB_FP64, HSB_SPLIT_INT8, HSB_SPLIT_CRT, HSB_SPLIT_CRT_BF16


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1712_07206_amd import _native
    _native.lib()
    yield


def _full(M):
    return np.triu(M) + np.triu(M, 1).conj().T


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _poisoned(n):
    return torch.full((n, n), complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")


@pytest.mark.parametrize("precision,n_slices,sizes", [(0, 0, (1000, 300)), (3, 6, (1000, 300)), (4, 11, (600, 300)),
                                                      (5, 11, (400, 200))])
def test_static_forward_matches_forward_twice(precision, n_slices, sizes):
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    # sizes: the second call smaller, in a scratch left dirty by the first
    b = HSBuilder.from_case(make_case(1, n_g=sizes[0]), max_ng=sizes[0], precision=precision, n_slices=n_slices)
    for n_g in sizes:
        case = make_case(1, n_g=n_g)
        need = b.workspace_bytes(N.HSB_MODE_FORWARD, [n_g])
        assert need <= N.HSB_STATIC_SCRATCH_BYTES, need
        print("static forward: cfg1 n_g=%d precision=%d workspace %d bytes" % (n_g, precision, need), flush=True)
        g, tau, T = case_tensors(case)
        Hs, Ss = _poisoned(n_g), _poisoned(n_g)
        b.forward_static(case["k_frac"], g, tau, T, Hs, Ss)
        Hw, Sw = _poisoned(n_g), _poisoned(n_g)
        b.forward(case["k_frac"], g, tau, T, Hw, Sw)
        torch.cuda.synchronize()
        Hs, Ss, Hw, Sw = (x.cpu().numpy() for x in (Hs, Ss, Hw, Sw))
        iu, il = np.triu_indices(n_g), np.tril_indices(n_g, -1)
        for got, ref in ((Hs, Hw), (Ss, Sw)):
            assert np.all(np.isfinite(got[iu]))
            assert np.all(np.isnan(got[il])), "strict lower triangle was written"
            assert np.array_equal(got[iu], ref[iu]), "static scratch result differs from the workspace result"
        Hr, Sr = o.hs(case)
        eh, es = _rel(_full(Hs), Hr), _rel(_full(Ss), Sr)
        print("  vs oracle: H %.3e S %.3e" % (eh, es), flush=True)
        assert eh <= TOL[precision] and es <= TOL[precision]


def test_static_forward_refuses_a_problem_beyond_the_scratch():
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    n_g = 3000
    case = make_case(2, n_g=n_g)  # stacked width 30976: about 4.5 GB of workspace
    b = HSBuilder.from_case(case)
    assert b.workspace_bytes(N.HSB_MODE_FORWARD, [n_g]) > N.HSB_STATIC_SCRATCH_BYTES
    g, tau, T = case_tensors(case)
    H, S = _poisoned(n_g), _poisoned(n_g)
    kf = (ctypes.c_double * 3)(*[float(x) for x in case["k_frac"]])
    code = N.lib().hsbuild_forward_static(b._h, kf, n_g, ctypes.c_void_p(g.data_ptr()),
                                          ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                          ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(S.data_ptr()), None)
    assert code == N.HSB_ERR_WORKSPACE
    assert "static scratch" in N.last_error(b._h)
    torch.cuda.synchronize()
    assert torch.isnan(H).all() and torch.isnan(S).all(), "outputs touched by a refused call"
