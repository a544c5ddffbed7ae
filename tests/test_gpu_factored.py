"""GPU parity of the type-factored H/S path (hsbuild_forward_factored) against
the oracle's Eqs. 4-5, through the C-ABI.

The factored contraction reaches the same H and S as the stacked one up to
FP64 rounding, so the bar is the FP64 path's: relative Frobenius error
<= 1e-12 for H and for S separately, and the strict lower triangle untouched.
"""
import numpy as np
import pytest
import torch

from flapw_cells import make_case, make_batch_case
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu

TOL_HS = 1e-12


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1712_07206_amd import _native
    _native.lib()
    yield


def _full(M):
    return np.triu(M) + np.triu(M, 1).conj().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _factored(case, poison=True, builder=None):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    n = case["n_g"]
    b = builder or HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    fill = complex(float("nan"), float("nan")) if poison else 0.0
    H = torch.full((n, n), fill, dtype=torch.complex128, device="cuda")
    S = H.clone()
    b.forward_factored(case["k_frac"], g, tau, T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


def _check_triangle(M):
    n = M.shape[0]
    assert np.all(np.isfinite(M[np.triu_indices(n)])), "upper triangle not fully written"
    assert np.all(np.isnan(M[np.tril_indices(n, -1)])), "strict lower triangle was written"


@pytest.mark.parametrize("idx,n_g", [(0, None), (1, 1), (1, 7), (1, 129), (1, 1000), (4, 800)])
def test_factored_matches_oracle(idx, n_g):
    case = make_case(idx, n_g=n_g)
    print("case", idx, "n_g", case["n_g"], flush=True)
    H, S = _factored(case)
    _check_triangle(H)
    _check_triangle(S)
    Hr, Sr = o.hs(case)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("factored vs oracle: H %.3e S %.3e" % (eh, es))
    assert eh <= TOL_HS and es <= TOL_HS


def test_factored_bench_cell_vs_oracle():
    """The bench cell (4 types x 32 atoms, l_max 10) at N_G = 3000."""
    case = make_case(2, n_g=3000)
    H, S = _factored(case)
    Hr, Sr = o.hs(case)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("factored cfg2@3000 vs oracle: H %.3e S %.3e" % (eh, es))
    assert eh <= TOL_HS and es <= TOL_HS


def test_factored_batch_cell_one_k():
    """One k-point of the 64-k cell (2 types x 16 atoms), its own N_G."""
    from flapw_cells import sub_case
    bc = make_batch_case(3, n_k=3)
    case = sub_case(bc, 2)
    H, S = _factored(case)
    Hr, Sr = o.hs(case)
    assert rel(_full(H), Hr) <= TOL_HS and rel(_full(S), Sr) <= TOL_HS


def test_factored_full_size_vs_fp64_path():
    """At the bench size (N_G = 12000) against the stacked FP64 path on the GPU,
    compared over the upper triangles without leaving the device."""
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(2)
    n = case["n_g"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H1 = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    S1 = torch.zeros_like(H1)
    b.forward(case["k_frac"], g, tau, T, H1, S1)
    b._ws = None
    H2 = torch.zeros_like(H1)
    S2 = torch.zeros_like(H1)
    b.forward_factored(case["k_frac"], g, tau, T, H2, S2)
    torch.cuda.synchronize()
    H1, H2, S1, S2 = torch.triu(H1), torch.triu(H2), torch.triu(S1), torch.triu(S2)
    eh = float(torch.linalg.norm(H2 - H1) / torch.linalg.norm(H1))
    es = float(torch.linalg.norm(S2 - S1) / torch.linalg.norm(S1))
    print("factored vs FP64 stacked at N_G=12000: H %.3e S %.3e" % (eh, es))
    assert eh <= TOL_HS and es <= TOL_HS


def test_factored_deterministic():
    case = make_case(1, n_g=700)
    H1, S1 = _factored(case, poison=False)
    H2, S2 = _factored(case, poison=False)
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2)


def test_factored_tile_orders_agree():
    """The tile order changes only which workgroup computes a tile."""
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder
    case = make_case(1, n_g=1500)
    b = HSBuilder.from_case(case)
    out = []
    for gr in (0, 3, 8):
        b.set_option(N.HSB_OPT_TILE_GROUP, gr)
        out.append(_factored(case, poison=False, builder=b))
    for H, S in out[1:]:
        assert np.array_equal(H, out[0][0]) and np.array_equal(S, out[0][1])


def test_factored_errors_launch_nothing():
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(1, n_g=300)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    n = case["n_g"]
    H = torch.full((n, n), 7.0, dtype=torch.complex128, device="cuda")
    S = H.clone()
    need = b.workspace_bytes(N.HSB_MODE_FACTORED, [n])
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(N.HSBuildError) as e:
        b.forward_factored(case["k_frac"], g, tau, T, H, S, ws=ws)
    assert e.value.code == N.HSB_ERR_WORKSPACE
    with pytest.raises(N.HSBuildError) as e:
        b.forward_factored(case["k_frac"], g, tau, T, H, H)
    assert e.value.code == N.HSB_ERR_ARG
    torch.cuda.synchronize()
    assert bool((H == 7.0).all()) and bool((S == 7.0).all())
