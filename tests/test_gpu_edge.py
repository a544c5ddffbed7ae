"""Edge configurations through every entry point, against the oracle:
the largest l_max (12, N_L = 169) and type count (16) the ABI accepts, one
atom per type; and an inversion-symmetric cell with a type that has no
atoms and an atom at the origin.  Bars as for the main paths: relative
Frobenius error <= 1e-12 (FP64 paths), <= 1e-10 (split, gradients)."""
import numpy as np
import pytest
import torch

from flapw_cells import make_case
from oracle import hs_oracle as o

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1712_07206_amd import _native
    _native.lib()
    yield


_cache = {}


def _oracle(idx):
    if idx not in _cache:
        case = make_case(idx)
        _cache[idx] = (case, o.hs(case))
    return _cache[idx]


def _full(M):
    return np.triu(M) + np.triu(M, 1).conj().T


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check(name, H, S, Hr, Sr, tol):
    eh, es = rel(_full(H), Hr), rel(_full(S), Sr)
    print("%s: H %.3e S %.3e" % (name, eh, es), flush=True)
    assert eh <= tol and es <= tol


@pytest.mark.parametrize("idx", [7, 8])
def test_edge_forward_factored_hsdla(idx):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case, (Hr, Sr) = _oracle(idx)
    print("case", case["name"], flush=True)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H, S = b.forward(case["k_frac"], g, tau, T)
    _check("forward", H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-12)
    H, S = b.forward_factored(case["k_frac"], g, tau, T)
    _check("factored", H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-12)
    H, S = b.forward_hsdla(3, case["k_frac"], g, tau, T)
    _check("rocBLAS Alg. 3", H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-12)


def test_edge_real_with_empty_type():
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case, (Hr, Sr) = _oracle(8)
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    H, S = b.forward_real(case["k_frac"], g, tau, case["partner"], T)
    H, S = H.cpu().numpy(), S.cpu().numpy()
    eh = rel(np.triu(H) + np.triu(H, 1).T, Hr.real)
    es = rel(np.triu(S) + np.triu(S, 1).T, Sr.real)
    print("real: H %.3e S %.3e" % (eh, es))
    assert eh <= 1e-12 and es <= 1e-12


@pytest.mark.parametrize("prec_name", ["bf16", "int8"])
def test_edge_split_lmax12(prec_name):
    from paper_1712_07206_amd import HSB_SPLIT_BF16, HSB_SPLIT_INT8
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    prec, slices = {"bf16": (HSB_SPLIT_BF16, 5), "int8": (HSB_SPLIT_INT8, 6)}[prec_name]
    case, (Hr, Sr) = _oracle(7)
    b = HSBuilder.from_case(case, precision=prec, n_slices=slices)
    g, tau, T = case_tensors(case)
    H, S = b.forward(case["k_frac"], g, tau, T)
    _check("split %s x%d" % (prec_name, slices), H.cpu().numpy(), S.cpu().numpy(), Hr, Sr, 1e-10)


@pytest.mark.parametrize("idx", [7, 8])
def test_edge_backward(idx):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    case = make_case(idx)
    n = case["n_g"]
    rng = np.random.default_rng(11)
    def herm():
        z = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        return (z + z.conj().T) / (2.0 * n)
    Wm, Vm = herm(), herm()
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    gT, gtau = b.backward(case["k_frac"], g, tau, T, torch.as_tensor(Wm, device="cuda"),
                          torch.as_tensor(Vm, device="cuda"))
    rT, rtau = o.loss_gradients(case, Wm, Vm)
    eT = np.linalg.norm(gT.cpu().numpy() - rT) / np.linalg.norm(rT)
    etau = np.linalg.norm(gtau.cpu().numpy() - rtau) / np.linalg.norm(rtau)
    print("backward: grad_T %.3e grad_tau %.3e" % (eT, etau))
    assert eT <= 1e-10 and etau <= 1e-10
    if idx == 8:  # the type without atoms gets no gradient
        assert float(torch.abs(gT[1]).max()) == 0.0
