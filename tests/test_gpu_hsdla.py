"""GPU parity of the paper's own BLAS sequence on rocBLAS (hsbuild_forward_hsdla,
Alg. 3 and Alg. 1) against the oracle's Eqs. 4-5, through the C-ABI.

Same bar as the fused FP64 path: relative Frobenius error <= 1e-12 for H and
S separately.  Alg. 3 writes the upper triangles only; Alg. 1's H_AA step is a
general product, so its H is compared over the upper triangle.
"""
import numpy as np
import pytest
import torch

from flapw_cells import make_case
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


def _hsdla(case, algorithm):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    n = case["n_g"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    nan = complex(float("nan"), float("nan"))
    H = torch.full((n, n), nan if algorithm == 3 else 0.0, dtype=torch.complex128, device="cuda")
    S = torch.full((n, n), nan, dtype=torch.complex128, device="cuda")
    b.forward_hsdla(algorithm, case["k_frac"], g, tau, T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("algorithm", [3, 1])
@pytest.mark.parametrize("idx,n_g", [(0, None), (1, 7), (1, 1000)])
def test_hsdla_matches_oracle(algorithm, idx, n_g):
    case = make_case(idx, n_g=n_g)
    print("case", idx, "n_g", case["n_g"], "algorithm", algorithm, flush=True)
    H, S = _hsdla(case, algorithm)
    n = case["n_g"]
    assert np.all(np.isnan(S[np.tril_indices(n, -1)])), "S lower triangle written"
    if algorithm == 3:
        assert np.all(np.isnan(H[np.tril_indices(n, -1)])), "H lower triangle written"
    Hr, Sr = o.hs(case)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("hsdla alg %d vs oracle: H %.3e S %.3e" % (algorithm, eh, es))
    assert eh <= TOL_HS and es <= TOL_HS


def test_hsdla_bench_cell_vs_oracle():
    case = make_case(2, n_g=3000)
    H, S = _hsdla(case, 3)
    Hr, Sr = o.hs(case)
    assert rel(_full(H), Hr) <= TOL_HS and rel(_full(S), Sr) <= TOL_HS


def test_hsdla_rejects_unknown_algorithm():
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(0)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    with pytest.raises(N.HSBuildError) as e:
        b.forward_hsdla(2, case["k_frac"], g, tau, T)
    assert e.value.code == N.HSB_ERR_ARG
