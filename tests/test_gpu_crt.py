"""Residue (Chinese remainder) form of the split contraction, HSB_SPLIT_CRT:
operand columns scaled by powers of two and rounded to Gaussian integers,
their residues modulo coprime moduli multiplied on the int8 matrix cores,
the integer products recovered in FP64.  Bar: relative Frobenius error
<= 1e-10 for H and for S against the oracle at 11 moduli, lower triangle
untouched; exact (to FP64 rounding) where the scaled inputs are integers."""
import numpy as np
import pytest
import torch

from flapw_cells import at_k, make_case, shell_sizes
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-10
N_MOD = 11


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    yield


_cache = {}


def oracle(idx, n_g):
    if (idx, n_g) not in _cache:
        case = make_case(idx, n_g=n_g)
        _cache[(idx, n_g)] = (case, o.hs(case))
    return _cache[(idx, n_g)]


def _full(M):
    return np.triu(M) + np.triu(M, 1).conj().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _crt(case, n_mod=N_MOD, poison=True, waves=None, precision=None):
    from paper_1712_07206_amd import HSB_SPLIT_CRT
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    b = HSBuilder.from_case(case, precision=HSB_SPLIT_CRT if precision is None else precision, n_slices=n_mod)
    if waves is not None:
        b.set_option(N.HSB_OPT_HS_WAVES, waves)
    g, tau, T = case_tensors(case)
    n = case["n_g"]
    print("residue form: N_G %d, %d atoms, %d moduli, waves %s" % (n, case["n_atoms"], n_mod, waves), flush=True)
    fill = complex(float("nan"), float("nan")) if poison else 0.0
    H = torch.full((n, n), fill, dtype=torch.complex128, device="cuda")
    S = H.clone()
    b.forward(case["k_frac"], g, tau, T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("idx,n_g", [(0, None), (1, 1), (1, 7), (1, 129), (1, 1000), (2, 3000), (4, 800), (7, None),
                                     (8, None)])
def test_crt_matches_oracle(idx, n_g):
    case, (Hr, Sr) = oracle(idx, n_g)
    H, S = _crt(case)
    n = case["n_g"]
    il = np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle was written"
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("residue form idx %d N_G %d: rel err H %.3e S %.3e" % (idx, n, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


@pytest.mark.parametrize("waves", [4, 8])
@pytest.mark.parametrize("idx,n_g", [(1, 129), (2, 3000)])
def test_crt_wave_layouts_match_oracle_and_each_other(idx, n_g, waves):
    """Both contraction layouts (8 waves of 64 x 64, 4 waves of 128 x 64) against the
    oracle, and bitwise against each other (the int32 sums are exact)."""
    case, (Hr, Sr) = oracle(idx, n_g)
    H, S = _crt(case, waves=waves)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("residue form %d waves idx %d N_G %d: H %.3e S %.3e" % (waves, idx, n_g, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT
    H2, S2 = _crt(case, waves=12 - waves)
    iu = np.triu_indices(case["n_g"])
    assert np.array_equal(H[iu], H2[iu]) and np.array_equal(S[iu], S2[iu])


def test_crt_error_falls_with_moduli():
    """Each modulus adds log2(m)/2 > 3.4 bits to both operands: the error falls by more
    than 8x per modulus (8 to 13, the largest count); 11 moduli meet the bar."""
    case, (Hr, Sr) = oracle(1, 1000)
    errs = {}
    for k in range(8, 14):
        H, S = _crt(case, n_mod=k, poison=False)
        errs[k] = max(rel(_full(H), Hr), rel(_full(S), Sr))
    print("residue form error by moduli 8..13:", errs)
    for k in range(8, 13):
        assert errs[k] / errs[k + 1] > 8.0, errs
    assert errs[8] > TOL_SPLIT  # too few moduli miss the bar: the sweep measures something
    assert errs[11] <= TOL_SPLIT and errs[13] <= 1e-13


@pytest.mark.parametrize("bits,tol", [(30, 1e-14), (50, 2.0 ** -32)])
def test_crt_on_few_bit_inputs(bits, tol):
    """Coefficients with `bits` significant bits per column scale, lambda = 1, T = 1
    (so H = S = W^H W, by hsbuild_forward_coefficients).  At 11 moduli a column is
    scaled to a 2-norm near 2^40.9, about 2^35 per entry at this stacked width
    (2592), so 30-bit inputs become integers exactly and the residues give the exact
    integer product: the result is the FP64 product to FP64 rounding.  50-bit inputs
    are rounded by at most 2^-35.7 of their column's norm, which bounds the error."""
    from paper_1712_07206_amd import HSB_SPLIT_CRT
    from paper_1712_07206_amd.hsbuild import HSBuilder
    case = dict(make_case(1, n_g=640))
    n, n_at, n_l = 640, case["n_atoms"], case["n_l"]
    case["udot_norm2"] = np.ones_like(case["udot_norm2"])
    m = 2 * n_l
    case["T"] = np.stack([np.eye(m, dtype=np.complex128)] * case["n_types"])
    rng = np.random.default_rng(9)
    e = rng.integers(-3, 4, n)
    mant = rng.integers(-(2 ** bits) + 1, 2 ** bits, size=(n_at, 2, n_l, n, 2)).astype(np.float64)
    coef = (mant[..., 0] + 1j * mant[..., 1]) * np.ldexp(1.0, e - bits)[None, None, None, :]
    b = HSBuilder.from_case(case, precision=HSB_SPLIT_CRT, n_slices=N_MOD)
    H, S = b.forward_from_coefficients(torch.as_tensor(coef, device="cuda"), torch.as_tensor(case["T"], device="cuda"))
    Sr = o.overlap(case, coef)
    eh, es = rel(_full(H.cpu().numpy()), Sr), rel(_full(S.cpu().numpy()), Sr)
    print("residue form on %d-bit inputs: rel err H %.3e S %.3e" % (bits, eh, es))
    assert eh <= tol and es <= tol


def test_crt_full_size_against_fp64_path():
    """Full-size workload (N_G = 12000, stacked width 30976) in the benchmark's launch
    configuration (11 moduli) against the FP64 MFMA path."""
    from paper_1712_07206_amd import HSB_SPLIT_CRT
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors, hermitian_full
    case = make_case(2)
    g, tau, T = case_tensors(case)
    b64 = HSBuilder.from_case(case)
    H64, S64 = b64.forward(case["k_frac"], g, tau, T)
    H64, S64 = hermitian_full(H64), hermitian_full(S64)
    b64.close()
    del b64
    torch.cuda.empty_cache()
    print("residue form at full size", flush=True)
    bs = HSBuilder.from_case(case, precision=HSB_SPLIT_CRT, n_slices=N_MOD)
    Hs, Ss = bs.forward(case["k_frac"], g, tau, T)
    Hs, Ss = hermitian_full(Hs), hermitian_full(Ss)
    eh = (torch.linalg.norm(Hs - H64) / torch.linalg.norm(H64)).item()
    es = (torch.linalg.norm(Ss - S64) / torch.linalg.norm(S64)).item()
    print("full-size residue form vs fp64: H %.3e S %.3e" % (eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


def _wide_case(n_g, extra_per_type):
    """The bench cell with `extra_per_type` more atoms of every type at seeded
    positions: 288 atoms give 69696 stacked rows, past the 65536-row window after
    which the contraction reduces its int32 sums modulo m."""
    case = dict(make_case(2, n_g=n_g))
    rng = np.random.default_rng(20171211)
    types, taus = [], []
    for t in range(case["n_types"]):
        old = case["tau"][case["atom_type"] == t]
        new = rng.uniform(0.0, 1.0, size=(extra_per_type, 3)) @ case["lattice"]
        types.append(np.full(len(old) + extra_per_type, t, dtype=case["atom_type"].dtype))
        taus.append(np.concatenate([old, new]))
    case["atom_type"] = np.concatenate(types)
    case["tau"] = np.concatenate(taus)
    case["n_atoms"] = len(case["atom_type"])
    return case


@pytest.mark.parametrize("waves", [4, 8])
def test_crt_past_the_reduction_window(waves):
    """69696 stacked rows: the 8-wave layout reduces its sums modulo m after 65536 rows;
    the 4-wave layout, which has no reduction, stays exact up to 131072 rows."""
    case = _wide_case(96, 40)
    assert 65536 < 2 * case["n_atoms"] * case["n_l"] <= 131072
    Hr, Sr = o.hs(case)
    H, S = _crt(case, waves=waves)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("residue form (%d waves) at stacked width %d: rel err H %.3e S %.3e" % (
        waves, 2 * case["n_atoms"] * case["n_l"], eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


def _real_crt(case, poison=True, waves=None, precision=None):
    from paper_1712_07206_amd import HSB_SPLIT_CRT
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    b = HSBuilder.from_case(case, precision=HSB_SPLIT_CRT if precision is None else precision, n_slices=N_MOD)
    if waves is not None:
        b.set_option(N.HSB_OPT_HS_WAVES, waves)
    g, tau, T = case_tensors(case)
    n = case["n_g"]
    print("real residue form: N_G %d, %d atoms" % (n, case["n_atoms"]), flush=True)
    fill = float("nan") if poison else 0.0
    H = torch.full((n, n), fill, dtype=torch.float64, device="cuda")
    S = H.clone()
    b.forward_real(case["k_frac"], g, tau, case["partner"], T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("idx,n_g", [(5, None), (5, 1), (5, 7), (5, 300), (6, 3000)])
def test_real_crt_matches_oracle(idx, n_g):
    case, (Hr, Sr) = oracle(idx, n_g)
    H, S = _real_crt(case)
    n = case["n_g"]
    il = np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle was written"
    eh = rel(np.triu(H) + np.triu(H, 1).T, Hr.real)
    es = rel(np.triu(S) + np.triu(S, 1).T, Sr.real)
    print("real residue form idx %d N_G %d: H %.3e S %.3e" % (idx, n, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


def test_crt_at_gamma():
    """k on a lattice point (K = 0 in the basis, K_hat = z, only l = 0 there), at a
    closed-shell basis size."""
    base = make_case(1, n_g=123)
    sizes = shell_sizes(base["lattice"], np.zeros(3), 200)
    assert 123 in sizes
    case = at_k(base, np.zeros(3), n_g=123)
    Hr, Sr = o.hs(case)
    H, S = _crt(case)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("residue form at Gamma: H %.3e S %.3e" % (eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


def test_crt_is_reproducible():
    case, _ = oracle(1, 300)
    H1, S1 = _crt(case, poison=False)
    H2, S2 = _crt(case, poison=False)
    assert np.array_equal(H1, H2) and np.array_equal(S1, S2)


@pytest.mark.parametrize("waves", [4, 8])
def test_crt_stacked_widths_shorter_than_the_copy_ring(waves):
    """Stacked widths of one, two and three 64-row chunks, fewer than the four stages of
    the copy ring: a one-atom cell (50 rows), the two-atom cell (100) and the five-atom
    cell (160), and the real form of the five-atom cell (3 representatives, 96 rows: two
    chunks, each taken twice), against the oracle, in both contraction layouts."""
    base = make_case(0)
    one = dict(base)
    one["atom_type"], one["tau"], one["n_atoms"] = base["atom_type"][:1], base["tau"][:1], 1
    for case in (one, base, make_case(8)):
        Hr, Sr = o.hs(case)
        H, S = _crt(case, waves=waves)
        eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
        print("residue form (%d waves), stacked width %d: H %.3e S %.3e" % (
            waves, 2 * case["n_atoms"] * case["n_l"], eh, es))
        assert eh <= TOL_SPLIT and es <= TOL_SPLIT
    rcase, (Hr, Sr) = oracle(8, None)
    H, S = _real_crt(rcase, waves=waves)
    eh = rel(np.triu(H) + np.triu(H, 1).T, Hr.real)
    es = rel(np.triu(S) + np.triu(S, 1).T, Sr.real)
    print("real residue form (%d waves), five-atom cell: H %.3e S %.3e" % (waves, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


@pytest.mark.parametrize("kind", ["bf16", "fp16"])
@pytest.mark.parametrize("idx,n_g", [(0, None), (1, 129), (1, 1000), (8, None), (2, 3000)])
def test_crt_16bit_forms_bitwise_equal_to_byte_form(kind, idx, n_g):
    """The residues as bfloat16 or half integers on the 16-bit matrix cores, FP32 sums reduced
    modulo m every 1024 stacked rows (the 16-atom cell has 2592, the bench cell at N_G 3000
    30976): the residues are the same integers, so H and S equal the byte form's bitwise,
    and the oracle's bar holds."""
    from paper_1712_07206_amd import HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16
    prec = HSB_SPLIT_CRT_BF16 if kind == "bf16" else HSB_SPLIT_CRT_FP16
    case, (Hr, Sr) = oracle(idx, n_g)
    H8, S8 = _crt(case)
    H, S = _crt(case, precision=prec)
    n = case["n_g"]
    iu, il = np.triu_indices(n), np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle was written"
    assert np.array_equal(H[iu], H8[iu]) and np.array_equal(S[iu], S8[iu])
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("residue form (%s) idx %d N_G %d: rel err H %.3e S %.3e" % (kind, idx, n, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


@pytest.mark.parametrize("kind", ["bf16", "fp16"])
def test_real_crt_16bit_forms_bitwise_equal_to_byte_form(kind):
    """Real-symmetric form (both products in one FP32 sum, two stages per chunk) at N_G 300
    and on the full inversion-symmetric cell at N_G 3000."""
    from paper_1712_07206_amd import HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16
    prec = HSB_SPLIT_CRT_BF16 if kind == "bf16" else HSB_SPLIT_CRT_FP16
    for idx, n_g in ((5, 300), (6, 3000)):
        case, (Hr, Sr) = oracle(idx, n_g)
        H8, S8 = _real_crt(case)
        H, S = _real_crt(case, precision=prec)
        iu = np.triu_indices(case["n_g"])
        assert np.array_equal(H[iu], H8[iu]) and np.array_equal(S[iu], S8[iu])
        eh = rel(np.triu(H) + np.triu(H, 1).T, Hr.real)
        es = rel(np.triu(S) + np.triu(S, 1).T, Sr.real)
        print("real residue form (%s) idx %d N_G %d: H %.3e S %.3e" % (kind, idx, case["n_g"], eh, es))
        assert eh <= TOL_SPLIT and es <= TOL_SPLIT


@pytest.mark.parametrize("kind", ["bf16", "fp16"])
def test_crt_16bit_past_the_reduction_window(kind):
    """69696 stacked rows: the FP32 sums are reduced modulo m 68 times; bitwise equal to the
    byte form.  The 16-bit forms have the 8-wave layout only: asking for 4 waves runs it too."""
    from paper_1712_07206_amd import HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16
    prec = HSB_SPLIT_CRT_BF16 if kind == "bf16" else HSB_SPLIT_CRT_FP16
    case = _wide_case(96, 40)
    H8, S8 = _crt(case)
    iu = np.triu_indices(case["n_g"])
    for waves in (None, 4):
        H, S = _crt(case, precision=prec, waves=waves)
        assert np.array_equal(H[iu], H8[iu]) and np.array_equal(S[iu], S8[iu]), waves


def test_crt_default_layouts():
    """Defaults: the byte form takes the 4-wave layout, the 16-bit forms the 8-wave one; tile
    group 4 for all."""
    from paper_1712_07206_amd import HSB_SPLIT_CRT, HSB_SPLIT_CRT_BF16, HSB_SPLIT_CRT_FP16
    from paper_1712_07206_amd import _native as N
    from paper_1712_07206_amd.hsbuild import HSBuilder
    for prec, waves in ((HSB_SPLIT_CRT, 4), (HSB_SPLIT_CRT_BF16, 8), (HSB_SPLIT_CRT_FP16, 8)):
        b = HSBuilder.from_case(make_case(0), precision=prec, n_slices=N_MOD)
        assert b.get_option(N.HSB_OPT_HS_WAVES) == waves and b.get_option(N.HSB_OPT_TILE_GROUP) == 4
        b.close()
