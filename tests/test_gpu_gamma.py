"""Every entry point at k = 0, where the basis holds K = k + G = 0 (a k-point
on a lattice point, Sec. 2.1): the K_hat = z rule, the x = 0 branch of the
Bessel functions and the vanishing |K| j_l'(0) all run on the device.

Each test uses a closed-shell basis (the cut-off between two shells of
|k+G|, which the generator requires) and compares with the oracle: relative
Frobenius error over the mirrored matrices <= 1e-12 for the FP64 paths and
<= 1e-10 for the split forms, the same bound on max |entry error| / max |entry|,
and the strict lower triangle untouched (NaN-poisoned before the call)."""
import numpy as np
import pytest
import torch

from flapw_cells import at_k, make_batch_case, make_case, shell_sizes, sub_case
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu

GAMMA = np.zeros(3)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1712_07206_amd import _native
    _native.lib()
    yield


_cache = {}


def gamma(idx, n_g):
    """Workload idx at k = 0 with n_g basis functions (G = 0 first), and its oracle H, S."""
    key = (idx, n_g)
    if key not in _cache:
        case = at_k(make_case(idx, n_g=50), GAMMA, n_g)
        assert np.all(case["g"][0] == 0)
        _cache[key] = (case, o.hs(case))
    return _cache[key]


def _full(M):
    return np.triu(M) + np.triu(M, 1).conj().T


def _poisoned(n, dtype=torch.complex128):
    nan = complex(float("nan"), float("nan")) if dtype == torch.complex128 else float("nan")
    return torch.full((n, n), nan, dtype=dtype, device="cuda")


def _check(name, H, S, Hr, Sr, tol, real=False):
    """H, S: upper triangles from the device (lower triangle must still be NaN)."""
    n = H.shape[0]
    il = np.tril_indices(n, -1)
    iu = np.triu_indices(n)
    for M in (H, S):
        assert np.all(np.isfinite(M[iu])), name + ": upper triangle not fully written"
        assert np.all(np.isnan(M[il])), name + ": strict lower triangle was written"
    if real:
        Hf, Sf = np.triu(H) + np.triu(H, 1).T, np.triu(S) + np.triu(S, 1).T
        Hr, Sr = Hr.real, Sr.real
    else:
        Hf, Sf = _full(H), _full(S)
    fh = np.linalg.norm(Hf - Hr) / np.linalg.norm(Hr)
    fs = np.linalg.norm(Sf - Sr) / np.linalg.norm(Sr)
    mh = np.abs(Hf - Hr).max() / np.abs(Hr).max()
    ms = np.abs(Sf - Sr).max() / np.abs(Sr).max()
    print("%s: Frobenius H %.3e S %.3e, max-entry H %.3e S %.3e" % (name, fh, fs, mh, ms), flush=True)
    assert fh <= tol and fs <= tol and mh <= tol and ms <= tol
    # the K = 0 row carries only l = 0: it is checked on its own as well
    assert np.abs(Hf[0] - Hr[0]).max() <= tol * np.abs(Hr).max()
    assert np.abs(Sf[0] - Sr[0]).max() <= tol * np.abs(Sr).max()


@pytest.mark.parametrize("idx,n_g", [(0, 123), (1, 123)])
def test_gamma_coefficients(idx, n_g):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case, _ = gamma(idx, n_g)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    got = b.coefficients(case["k_frac"], g, tau).cpu().numpy()
    ref = o.coefficients(case)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("coefficients at k = 0:", err)
    assert err <= 1e-13
    # K = 0 column: only L = 00 is nonzero, and exactly zero elsewhere
    assert np.all(got[:, :, 1:, 0] == 0.0)
    np.testing.assert_allclose(got[:, :, 0, 0], ref[:, :, 0, 0], rtol=1e-14, atol=0)


@pytest.mark.parametrize("idx,n_g", [(0, 123), (1, 123), (2, 251)])
def test_gamma_forward_and_factored(idx, n_g):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case, (Hr, Sr) = gamma(idx, n_g)
    print("case", case["name"], "at k = 0, N_G", n_g, flush=True)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H, S = _poisoned(n_g), _poisoned(n_g)
    b.forward(GAMMA, g, tau, T, H, S)
    _check("forward", H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-12)
    H, S = _poisoned(n_g), _poisoned(n_g)
    b.forward_factored(GAMMA, g, tau, T, H, S)
    _check("factored", H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-12)
    H, S = _poisoned(n_g), _poisoned(n_g)
    b.forward_hsdla(3, GAMMA, g, tau, T, H, S)
    _check("rocBLAS Alg. 3", H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-12)


@pytest.mark.parametrize("prec_name,slices", [("int8", 6), ("bf16", 5), ("fp16", 5)])
def test_gamma_split(prec_name, slices):
    from paper_1712_07206_amd import HSB_SPLIT_BF16, HSB_SPLIT_FP16, HSB_SPLIT_INT8
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    prec = {"int8": HSB_SPLIT_INT8, "bf16": HSB_SPLIT_BF16, "fp16": HSB_SPLIT_FP16}[prec_name]
    case, (Hr, Sr) = gamma(1, 123)
    b = HSBuilder.from_case(case, precision=prec, n_slices=slices)
    g, tau, T = case_tensors(case)
    H, S = _poisoned(123), _poisoned(123)
    b.forward(GAMMA, g, tau, T, H, S)
    _check("split %s x%d" % (prec_name, slices), H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-10)


@pytest.mark.parametrize("prec_name", ["fp64", "int8"])
def test_gamma_real_symmetric(prec_name):
    """The inversion-symmetric cell at k = 0 (its atom at the origin included)."""
    from paper_1712_07206_amd import HSB_FP64, HSB_SPLIT_INT8
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case, (Hr, Sr) = gamma(5, 123)
    prec, slices, tol = (HSB_FP64, 0, 1e-12) if prec_name == "fp64" else (HSB_SPLIT_INT8, 6, 1e-10)
    b = HSBuilder.from_case(case, precision=prec, n_slices=slices)
    g, tau, T = case_tensors(case)
    H, S = _poisoned(123, torch.float64), _poisoned(123, torch.float64)
    b.forward_real(GAMMA, g, tau, case["partner"], T, H, S)
    assert np.abs(Hr.imag).max() <= 1e-13 * np.abs(Hr).max()
    _check("real %s" % prec_name, H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, tol, real=True)


def test_gamma_backward():
    """Gradients at k = 0 on the loss workload's cell against the oracle's (per-atom
    route); the K = 0 column contributes nothing to the position gradient."""
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = at_k(make_case(4, n_g=50), GAMMA, 123)
    n = case["n_g"]
    rng = np.random.default_rng(12)

    def herm():
        z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        return (z + z.conj().T) / (2.0 * n)

    Wm, Vm = herm(), herm()
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    gT, gtau = b.backward(GAMMA, g, tau, T, torch.as_tensor(Wm, device="cuda"), torch.as_tensor(Vm, device="cuda"))
    rT, rtau = o.loss_gradients(case, Wm, Vm)
    eT = np.linalg.norm(gT.cpu().numpy() - rT) / np.linalg.norm(rT)
    etau = np.linalg.norm(gtau.cpu().numpy() - rtau) / np.linalg.norm(rtau)
    print("backward at k = 0: grad_T %.3e grad_tau %.3e" % (eT, etau))
    assert eT <= 1e-10 and etau <= 1e-10


def test_gamma_in_batch():
    """A batch whose first k-point is k = 0 (closed-shell basis) among ordinary ones:
    the k = 0 block against the oracle, every block bitwise against single-k forwards."""
    from paper_1712_07206_amd.hsbuild import HSBuilder
    base = make_batch_case(3, n_k=3)
    n0 = [s for s in shell_sizes(base["lattice"], GAMMA, 400) if s >= 300][0]
    g0 = at_k(sub_case(base, 0), GAMMA, n0)["g"]
    kf = np.concatenate([GAMMA[None, :], base["k_frac"][1:]])
    gs = [g0] + list(base["g"][1:])
    b = HSBuilder.from_case(dict(base, n_g=np.array([len(x) for x in gs])))
    from paper_1712_07206_amd import _native as N
    b.set_option(N.HSB_OPT_SPLIT_K, 0)  # single-k forwards in the one-pass form the batch equals bitwise
    tau = torch.as_tensor(base["tau"], device="cuda")
    T = torch.as_tensor(base["T"], device="cuda")
    gl = [torch.as_tensor(x, device="cuda") for x in gs]
    H, S, off = b.batch(kf, gl, tau, T)
    torch.cuda.synchronize()
    Hc, Sc = H.cpu().numpy(), S.cpu().numpy()
    for k in range(3):
        n = len(gs[k])
        Hk = Hc[int(off[k]): int(off[k]) + n * n].reshape(n, n)
        Sk = Sc[int(off[k]): int(off[k]) + n * n].reshape(n, n)
        h1, s1 = b.forward(kf[k], gl[k], tau, T)
        iu = np.triu_indices(n)
        assert np.array_equal(Hk[iu], h1.cpu().numpy()[iu]) and np.array_equal(Sk[iu], s1.cpu().numpy()[iu]), k
        if k == 0:
            case0 = dict(sub_case(base, 0), k_frac=GAMMA.copy(), g=g0, n_g=n)
            Hr, Sr = o.hs(case0)
            eh = np.linalg.norm(_full(Hk) - Hr) / np.linalg.norm(Hr)
            es = np.linalg.norm(_full(Sk) - Sr) / np.linalg.norm(Sr)
            mh = np.abs(_full(Hk) - Hr).max() / np.abs(Hr).max()
            print("batch k = 0 (N_G %d): H %.3e S %.3e max-entry H %.3e" % (n, eh, es, mh))
            assert eh <= 1e-12 and es <= 1e-12 and mh <= 1e-12
