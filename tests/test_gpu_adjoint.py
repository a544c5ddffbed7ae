"""GPU adjoint (hsbuild_backward) against the oracle's gradient and against
central differences of the GPU forward.

Loss L = Re tr(W H) + Re tr(V S) with the workload's Hermitian W, V, so
dL/dH = W^H = W and dL/dS = V (torch convention).  Tolerances: <= 1e-10
norm-relative against the oracle gradient; <= 1e-7 against central
differences (tau step 1e-6 bohr, T step 1e-7)."""
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
    yield


def _setup(case):
    from paper_1712_07206_amd.hsbuild import HSBuilder, case_tensors
    b = HSBuilder.from_case(case)
    g, tau, T = case_tensors(case)
    Wm = torch.as_tensor(case["W"], device="cuda")
    Vm = torch.as_tensor(case["V"], device="cuda")
    return b, g, tau, T, Wm, Vm


def _loss(b, case, g, tau, T, Wm, Vm):
    from paper_1712_07206_amd.hsbuild import hermitian_full
    H, S = b.forward(case["k_frac"], g, tau, T)
    H = hermitian_full(H)
    S = hermitian_full(S)
    return float((torch.sum(Wm * H.transpose(0, 1)).real + torch.sum(Vm * S.transpose(0, 1)).real).item())


@pytest.mark.parametrize("n_g", [37, 129, 800])
def test_backward_matches_oracle_gradient(n_g):
    """One, two and seven 128-wide blocks of G (the padded W^T and gradients of
    the adjoint products are ragged at the first two)."""
    case = make_case(4, n_g=n_g)
    b, g, tau, T, Wm, Vm = _setup(case)
    gT, gtau = b.backward(case["k_frac"], g, tau, T, Wm, Vm)
    torch.cuda.synchronize()
    rT, rtau = o.loss_gradients(case, case["W"], case["V"])
    eT = np.linalg.norm(gT.cpu().numpy() - rT) / np.linalg.norm(rT)
    etau = np.linalg.norm(gtau.cpu().numpy() - rtau) / np.linalg.norm(rtau)
    print("adjoint vs oracle: grad_T %.3e grad_tau %.3e" % (eT, etau))
    assert eT <= 1e-10 and etau <= 1e-10


def test_backward_deterministic():
    case = make_case(4, n_g=500)
    b, g, tau, T, Wm, Vm = _setup(case)
    a1 = [x.cpu().numpy() for x in b.backward(case["k_frac"], g, tau, T, Wm, Vm)]
    a2 = [x.cpu().numpy() for x in b.backward(case["k_frac"], g, tau, T, Wm, Vm)]
    assert np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1], a2[1])


def test_backward_central_differences_full_size():
    """Full-size differentiation workload (64 atoms, N_L = 121, N_G = 6000)."""
    case = make_case(4)
    b, g, tau, T, Wm, Vm = _setup(case)
    gT, gtau = b.backward(case["k_frac"], g, tau, T, Wm, Vm)
    gtau = gtau.cpu().numpy()
    gT = gT.cpu().numpy()
    rng = np.random.default_rng(44)
    h = 1e-6
    picks = [(int(a), int(c)) for a, c in zip(rng.integers(0, case["n_atoms"], 6), rng.integers(0, 3, 6))]
    fd, an = [], []
    for a, c in picks:
        tp = tau.clone()
        tp[a, c] += h
        tm = tau.clone()
        tm[a, c] -= h
        fd.append((_loss(b, case, g, tp, T, Wm, Vm) - _loss(b, case, g, tm, T, Wm, Vm)) / (2 * h))
        an.append(gtau[a, c])
    fd, an = np.array(fd), np.array(an)
    err = np.abs(fd - an).max() / np.abs(gtau).max()
    print("tau FD max err (rel to max |grad|)", err, fd, an)
    assert err <= 1e-7
    # T: L is linear in T, so the central difference along a Hermitian direction is exact up to rounding
    m = T.shape[1]
    for _ in range(2):
        D = rng.normal(size=(case["n_types"], m, m)) + 1j * rng.normal(size=(case["n_types"], m, m))
        D = D + np.conj(np.transpose(D, (0, 2, 1)))
        Dt = torch.as_tensor(D, device="cuda")
        ht = 1e-7
        fdT = (_loss(b, case, g, tau, T + ht * Dt, Wm, Vm) - _loss(b, case, g, tau, T - ht * Dt, Wm, Vm)) / (2 * ht)
        pred = float(np.real(np.sum(np.conj(gT) * D)))
        print("T FD", fdT, pred)
        assert abs(fdT - pred) <= 1e-7 * abs(pred)


def test_backward_identities():
    """Euler identity (L_H linear in T) and the translation sum rule."""
    case = make_case(4, n_g=1000)
    b, g, tau, T, Wm, Vm = _setup(case)
    zero = torch.zeros_like(Vm)
    gT, _ = b.backward(case["k_frac"], g, tau, T, Wm, zero)
    lh = _loss(b, case, g, tau, T, Wm, zero)
    euler = float(torch.sum(torch.conj(gT) * T).real.item())
    assert abs(euler - lh) <= 1e-11 * abs(lh)
    _, gtau = b.backward(case["k_frac"], g, tau, T, Wm, Vm)
    from paper_1712_07206_amd.hsbuild import hermitian_full
    H, S = b.forward(case["k_frac"], g, tau, T)
    H = hermitian_full(H).cpu().numpy()
    S = hermitian_full(S).cpu().numpy()
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    M = case["W"].T * H + case["V"].T * S
    total = gtau.sum(0).cpu().numpy()
    for c in range(3):
        dk = kvec[None, :, c] - kvec[:, None, c]
        ref = float(np.real(np.sum(1j * dk * M)))
        assert abs(total[c] - ref) <= 1e-11 * np.abs(gtau.cpu().numpy()).max() * case["n_atoms"]


def test_autograd_function():
    from paper_1712_07206_amd.autograd import hs_build
    case = make_case(4, n_g=300)
    b, g, tau, T, Wm, Vm = _setup(case)
    tau_p = tau.clone().requires_grad_(True)
    T_p = T.clone().requires_grad_(True)
    H, S = hs_build(tau_p, T_p, b, case["k_frac"], g)
    L = torch.sum(Wm * H.transpose(0, 1)).real + torch.sum(Vm * S.transpose(0, 1)).real
    L.backward()
    rT, rtau = o.loss_gradients(case, case["W"], case["V"])
    assert np.linalg.norm(tau_p.grad.cpu().numpy() - rtau) <= 1e-10 * np.linalg.norm(rtau)
    assert np.linalg.norm(T_p.grad.cpu().numpy() - rT) <= 1e-10 * np.linalg.norm(rT)
