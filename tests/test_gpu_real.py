"""GPU parity of the real-symmetric path (hsbuild_forward_real) for
inversion-symmetric cells against the oracle's Eqs. 4-5, through the C-ABI.

On these cells the oracle's H and S are real (pinned on the CPU), so the bar
is the FP64 path's: relative Frobenius error <= 1e-12 of the real outputs
against the oracle's real parts, strict lower triangle untouched.
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
    return np.triu(M) + np.triu(M, 1).T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _real(case, partner=None, poison=True):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    n = case["n_g"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H = torch.full((n, n), float("nan") if poison else 0.0, dtype=torch.float64, device="cuda")
    S = H.clone()
    b.forward_real(case["k_frac"], g, tau, case["partner"] if partner is None else partner, T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("idx,n_g", [(5, None), (5, 1), (5, 7), (5, 300), (6, 3000)])
def test_real_matches_oracle(idx, n_g):
    case = make_case(idx, n_g=n_g)
    print("case", idx, "n_g", case["n_g"], flush=True)
    H, S = _real(case)
    n = case["n_g"]
    il = np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle written"
    assert np.all(np.isfinite(H[np.triu_indices(n)])) and np.all(np.isfinite(S[np.triu_indices(n)]))
    Hr, Sr = o.hs(case)
    eh, es = rel(_full(H), Hr.real), rel(_full(S), Sr.real)
    print("real path vs oracle: H %.3e S %.3e" % (eh, es))
    assert eh <= TOL_HS and es <= TOL_HS


def test_real_full_size_vs_complex_path():
    """At N_G = 12000 against hsbuild_forward's real parts, on the device."""
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(6)
    n = case["n_g"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    Hc = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    Sc = torch.zeros_like(Hc)
    b.forward(case["k_frac"], g, tau, T, Hc, Sc)
    b._ws = None
    Hr = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    Sr = torch.zeros_like(Hr)
    b.forward_real(case["k_frac"], g, tau, case["partner"], T, Hr, Sr)
    torch.cuda.synchronize()
    Hc, Sc = torch.triu(Hc), torch.triu(Sc)
    imag_h = float(torch.linalg.norm(Hc.imag) / torch.linalg.norm(Hc))
    eh = float(torch.linalg.norm(torch.triu(Hr) - Hc.real) / torch.linalg.norm(Hc.real))
    es = float(torch.linalg.norm(torch.triu(Sr) - Sc.real) / torch.linalg.norm(Sc.real))
    print("real vs complex path at N_G=12000: H %.3e S %.3e; |Im H|/|H| of the complex path %.3e" % (eh, es, imag_h))
    assert imag_h <= 1e-13
    assert eh <= TOL_HS and es <= TOL_HS


def test_real_deterministic():
    case = make_case(5)
    H1, S1 = _real(case, poison=False)
    H2, S2 = _real(case, poison=False)
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2)


def test_real_rejects_bad_partner_map():
    from paper_1712_07206_amd import _native as N
    case = make_case(5, n_g=50)
    bad = case["partner"].copy()
    bad[0], bad[2] = bad[2], bad[0]  # no longer an involution
    with pytest.raises(N.HSBuildError) as e:
        _real(case, partner=bad)
    assert e.value.code == N.HSB_ERR_ARG
    cross = np.arange(case["n_atoms"], dtype=np.int32)
    cross[0], cross[8] = 8, 0  # pairs atoms of different types
    with pytest.raises(N.HSBuildError) as e:
        _real(case, partner=cross)
    assert e.value.code == N.HSB_ERR_ARG


def test_real_wave_variants_bitwise_equal():
    """The 8-wave (128 x 128 tiles) and 4-wave (128 x 64 tiles) real kernels add
    the same products in the same order for every entry."""
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(5)
    n = case["n_g"]
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    out = []
    for wv in (8, 4):
        b.set_option(N.HSB_OPT_HS_WAVES, wv)
        H = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        S = torch.zeros_like(H)
        b.forward_real(case["k_frac"], g, tau, case["partner"], T, H, S)
        torch.cuda.synchronize()
        out.append((H.cpu().numpy(), S.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def _real_int8(case, poison=True):
    from paper_1712_07206_amd import HSB_SPLIT_INT8
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    n = case["n_g"]
    b = HSBuilder.from_case(case, precision=HSB_SPLIT_INT8, n_slices=6)
    g, tau, T = case_tensors(case)
    H = torch.full((n, n), float("nan") if poison else 0.0, dtype=torch.float64, device="cuda")
    S = H.clone()
    b.forward_real(case["k_frac"], g, tau, case["partner"], T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("idx,n_g", [(5, None), (5, 1), (5, 7), (5, 300), (6, 3000)])
def test_real_int8_split_matches_oracle(idx, n_g):
    """The int8 split form of the real path (6 slices of 7 bits): the split
    bar, relative Frobenius error <= 1e-10 against the oracle's real parts."""
    case = make_case(idx, n_g=n_g)
    print("case", idx, "n_g", case["n_g"], flush=True)
    H, S = _real_int8(case)
    n = case["n_g"]
    il = np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle written"
    Hr, Sr = o.hs(case)
    eh, es = rel(_full(H), Hr.real), rel(_full(S), Sr.real)
    print("real int8 split vs oracle: H %.3e S %.3e" % (eh, es))
    assert eh <= 1e-10 and es <= 1e-10


def test_real_rejects_16bit_split_handles():
    """The real path has FP64 and int8 forms only: a BF16 handle gets
    HSB_ERR_UNSUPPORTED before anything is enqueued."""
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(5, n_g=7)
    b = HSBuilder.from_case(case, precision=N.HSB_SPLIT_BF16, n_slices=5)
    g, tau, T = case_tensors(case)
    H = torch.zeros((7, 7), dtype=torch.float64, device="cuda")
    S = torch.zeros_like(H)
    with pytest.raises(N.HSBuildError) as err:
        b.forward_real(case["k_frac"], g, tau, case["partner"], T, H, S)
    assert err.value.code == N.HSB_ERR_UNSUPPORTED


def test_real_int8_full_size_vs_fp64_real():
    """Full size (N_G = 12000, the bench's inversion cell and launch
    configuration): the int8 form of the real path against the FP64 one, on
    the device, to the split bar."""
    from paper_1712_07206_amd import HSB_SPLIT_INT8
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(6)
    n = case["n_g"]
    g, tau, T = case_tensors(case)
    b = HSBuilder.from_case(case)
    H64 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    S64 = torch.zeros_like(H64)
    b.forward_real(case["k_frac"], g, tau, case["partner"], T, H64, S64)
    b.close()
    del b
    torch.cuda.empty_cache()
    bi = HSBuilder.from_case(case, precision=HSB_SPLIT_INT8, n_slices=6)
    H8 = torch.zeros_like(H64)
    S8 = torch.zeros_like(H64)
    bi.forward_real(case["k_frac"], g, tau, case["partner"], T, H8, S8)
    torch.cuda.synchronize()
    H64, S64, H8, S8 = torch.triu(H64), torch.triu(S64), torch.triu(H8), torch.triu(S8)
    eh = (torch.linalg.norm(H8 - H64) / torch.linalg.norm(H64)).item()
    es = (torch.linalg.norm(S8 - S64) / torch.linalg.norm(S64)).item()
    print("full-size real int8 vs fp64 real: H %.3e S %.3e" % (eh, es))
    assert eh <= 1e-10 and es <= 1e-10
