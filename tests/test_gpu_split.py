"""Split-precision (Ozaki slice) forward: BF16 and FP16 slices on MFMA with
FP32 accumulation, or int8 slices with exact int32 accumulation, FP64
recombination.  Bar: relative Frobenius error <= 1e-10 for H and for S against
the oracle (5 slices of 8 bits for BF16/FP16, 6 slices of 7 bits for int8)."""
import numpy as np
import pytest
import torch

from flapw_cells import make_case
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu

TOL_SPLIT = 1e-10


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


def _split(case, precision, slices, poison=True):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    b = HSBuilder.from_case(case, precision=precision, n_slices=slices)
    g, tau, T = case_tensors(case)
    n = case["n_g"]
    fill = complex(float("nan"), float("nan")) if poison else 0.0
    H = torch.full((n, n), fill, dtype=torch.complex128, device="cuda")
    S = H.clone()
    b.forward(case["k_frac"], g, tau, T, H, S)
    torch.cuda.synchronize()
    return H.cpu().numpy(), S.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _prec(name):
    from paper_1712_07206_amd import HSB_SPLIT_BF16, HSB_SPLIT_FP16, HSB_SPLIT_INT8
    return {"bf16": (HSB_SPLIT_BF16, 5), "fp16": (HSB_SPLIT_FP16, 5), "int8": (HSB_SPLIT_INT8, 6)}[name]


@pytest.mark.parametrize("prec_name", ["bf16", "fp16", "int8"])
@pytest.mark.parametrize("idx,n_g", [(0, None), (1, 1), (1, 7), (1, 129), (1, 1000), (2, 3000), (4, 800)])
def test_split_matches_oracle(prec_name, idx, n_g):
    prec, slices = _prec(prec_name)
    case, (Hr, Sr) = oracle(idx, n_g)
    H, S = _split(case, prec, slices)
    n = case["n_g"]
    il = np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle was written"
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("split %s idx %d N_G %d: rel err H %.3e S %.3e" % (prec_name, idx, n, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


@pytest.mark.parametrize("prec_name", ["bf16", "fp16", "int8"])
def test_split_error_falls_with_slices(prec_name):
    prec, _ = _prec(prec_name)
    case, (Hr, Sr) = oracle(1, 1000)
    errs = []
    for s in (3, 4, 5, 6):
        H, S = _split(case, prec, s, poison=False)
        errs.append(max(rel(_full(H), Hr), rel(_full(S), Sr)))
    print("%s error by slice count 3..6:" % prec_name, errs)
    assert errs[0] > errs[1] > errs[2] > errs[3]
    if prec_name in ("bf16", "fp16"):  # 8-bit slices: about 2^8 per added slice
        assert all(a / b > 60 for a, b in zip(errs, errs[1:])), errs
        assert errs[0] < 1e-4 and errs[2] < TOL_SPLIT and errs[3] < 1e-12
    else:  # 7-bit slices: about 2^7 per added slice
        assert all(a / b > 30 for a, b in zip(errs, errs[1:])), errs
        assert errs[0] < 1e-4 and errs[3] < TOL_SPLIT


@pytest.mark.parametrize("prec_name", ["bf16", "int8"])
def test_split_full_size_against_fp64_path(prec_name):
    """Full-size workload (N_G = 12000, stacked width 30976) in the benchmark's
    launch configuration (BF16 with 5 slices, int8 with 6) against the FP64 MFMA
    path."""
    prec, slices = _prec(prec_name)
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors, hermitian_full
    case = make_case(2)
    g, tau, T = case_tensors(case)
    b64 = HSBuilder.from_case(case)
    H64, S64 = b64.forward(case["k_frac"], g, tau, T)
    H64, S64 = hermitian_full(H64), hermitian_full(S64)
    b64.close()
    del b64
    torch.cuda.empty_cache()
    bs = HSBuilder.from_case(case, precision=prec, n_slices=slices)
    Hs, Ss = bs.forward(case["k_frac"], g, tau, T)
    Hs, Ss = hermitian_full(Hs), hermitian_full(Ss)
    eh = (torch.linalg.norm(Hs - H64) / torch.linalg.norm(H64)).item()
    es = (torch.linalg.norm(Ss - S64) / torch.linalg.norm(S64)).item()
    print("full-size split %s vs fp64: H %.3e S %.3e" % (prec_name, eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT


def _wide_case(n_g, extra_per_type):
    """The bench cell with `extra_per_type` more atoms of every type (seeded
    positions in the cell): 160 atoms give 38720 stacked rows, past the int8
    kernel's 32768-row window between flushes of its int32 level sums."""
    case = dict(make_case(2, n_g=n_g))
    rng = np.random.default_rng(20171209)
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


@pytest.mark.parametrize("prec_name", ["int8", "bf16"])
def test_split_past_the_int8_flush_window(prec_name):
    """Stacked width 38720 (two int8 flush windows, the second ragged) against the oracle."""
    prec, slices = _prec(prec_name)
    case = _wide_case(96, 8)
    assert 2 * case["n_atoms"] * case["n_l"] > 32768
    Hr, Sr = o.hs(case)
    H, S = _split(case, prec, slices)
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("split %s at stacked width %d: rel err H %.3e S %.3e" % (prec_name, 2 * case["n_atoms"] * case["n_l"], eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT



def _wide_inversion_case(n_g, extra_pairs_per_type):
    """The inversion-symmetric cell of the bench shape with `extra_pairs_per_type` more
    inversion pairs (tau, -tau) of every type at seeded positions: 136 representatives
    and more put the real path's stacked width past the int8 kernel's 32768-row window."""
    case = dict(make_case(6, n_g=n_g))
    rng = np.random.default_rng(20171210)
    types, taus, partner = [], [], []
    for t in range(case["n_types"]):
        idx = np.nonzero(case["atom_type"] == t)[0]
        base = len(taus)
        for a in idx:  # the old pairs keep their partners, shifted to the new numbering
            partner.append(base + int(case["partner"][a]) - int(idx[0]))
            taus.append(case["tau"][a])
            types.append(t)
        for _ in range(extra_pairs_per_type):
            f = rng.uniform(0.0, 1.0, 3) @ case["lattice"]
            i = len(taus)
            taus.extend([f, -f])
            partner.extend([i + 1, i])
            types.extend([t, t])
    case["atom_type"] = np.asarray(types, dtype=np.int32)
    case["tau"] = np.ascontiguousarray(np.asarray(taus))
    case["partner"] = np.asarray(partner, dtype=np.int32)
    case["n_atoms"] = len(types)
    return case


def test_real_int8_past_the_flush_window():
    """Real-symmetric int8 split form with 136 representatives (stacked width 32912 >
    32768): the second flush adds into the outputs the first one wrote."""
    from paper_1712_07206_amd import HSB_SPLIT_INT8
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = _wide_inversion_case(96, 18)
    p = case["partner"]
    assert np.all(p[p] == np.arange(case["n_atoms"]))
    n_rep = int(np.sum(p >= np.arange(case["n_atoms"])))
    assert 2 * n_rep * case["n_l"] > 32768
    Hr, Sr = o.hs(case)
    assert np.abs(Hr.imag).max() <= 1e-12 * np.abs(Hr).max()
    b = HSBuilder.from_case(case, precision=HSB_SPLIT_INT8, n_slices=6)
    g, tau, T = case_tensors(case)
    n = case["n_g"]
    H = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    S = H.clone()
    b.forward_real(case["k_frac"], g, tau, case["partner"], T, H, S)
    H, S = H.cpu().numpy(), S.cpu().numpy()
    il = np.tril_indices(n, -1)
    assert np.all(np.isnan(H[il])) and np.all(np.isnan(S[il])), "strict lower triangle was written"
    eh = rel(np.triu(H) + np.triu(H, 1).T, Hr.real)
    es = rel(np.triu(S) + np.triu(S, 1).T, Sr.real)
    print("real int8 at stacked width %d: rel err H %.3e S %.3e" % (2 * n_rep * case["n_l"], eh, es))
    assert eh <= TOL_SPLIT and es <= TOL_SPLIT
