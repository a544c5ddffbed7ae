"""Planted mistakes in the oracle (CPU only) must each fail at least one pin.

Each mutation replaces one oracle function by a plausible wrong variant
(a dropped conjugate, factor i^l or term, a wrong sign, a swapped pair, a
transposed operand, a wrong normalisation), then the pin checks are run: the
unmutated oracle passes all of them, every mutant fails at least one.
"""
import numpy as np
import pytest
from scipy import special

from flapw_cells import at_k, make_case, perturb_positions
from oracle import hs_oracle as o


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def pin_plane_wave(mod):
    """Muffin-tin expansion = plane wave on the sphere (l_max 14, |K|R <= 1)."""
    base = make_case(0, n_g=256)
    l_max = 14
    case = dict(base, l_max=l_max)
    rng = np.random.default_rng(7)
    case["radial"] = rng.uniform(0.5, 1.5, (1, l_max + 1, 4))
    kvec = mod.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    keep = np.linalg.norm(kvec, axis=1) * case["r_mt"][0] <= 1.0
    coef = mod.coefficients(case, g=case["g"][keep])
    kvec = kvec[keep]
    R = case["r_mt"][0]
    pts = rng.normal(size=(12, 3))
    pts /= np.linalg.norm(pts, axis=1)[:, None]
    th = np.arccos(pts[:, 2])
    ph = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi)
    Yp = np.stack([special.sph_harm_y(l, m, th, ph) for l in range(l_max + 1) for m in range(-l, l + 1)])
    u = np.concatenate([[case["radial"][0, l, 0]] * (2 * l + 1) for l in range(l_max + 1)])
    ud = np.concatenate([[case["radial"][0, l, 2]] * (2 * l + 1) for l in range(l_max + 1)])
    err = 0.0
    for a in range(len(case["tau"])):
        val = (coef[a, 0] * u[:, None] + coef[a, 1] * ud[:, None]).T @ Yp
        pw = np.exp(1j * kvec @ (case["tau"][a][None, :] + R * pts).T) / np.sqrt(case["omega"])
        err = max(err, float(np.abs(val - pw).max()))
    return err <= 1e-12


def pin_matching(mod):
    kn = np.linspace(0.3, 4.0, 20)
    radial = np.random.default_rng(3).uniform(0.5, 1.5, (1, 2, 4))
    a, b = mod.matching(kn, np.array([1.7]), radial)
    x = kn * 1.7
    j0, dj0 = np.sin(x) / x, (x * np.cos(x) - np.sin(x)) / x ** 2
    u, du, ud, dud = radial[0, 0]
    return (np.abs(a[0, 0] * u + b[0, 0] * ud - j0).max() < 1e-12
            and np.abs(a[0, 0] * du + b[0, 0] * dud - kn * dj0).max() < 1e-12)


def _legendre(case, kvec, a, b, weights):
    kn = np.linalg.norm(kvec, axis=1)
    khat = kvec / kn[:, None]
    cosg = np.clip(khat @ khat.T, -1, 1)
    out = np.zeros((len(kvec), len(kvec)), dtype=np.complex128)
    for at, tau in enumerate(case["tau"]):
        t = int(case["atom_type"][at])
        ph = np.exp(1j * kvec @ tau)
        acc = sum((2 * l + 1) * special.eval_legendre(l, cosg) * weights(t, l, a[t, l], b[t, l])
                  for l in range(case["l_max"] + 1))
        out += np.conj(ph)[:, None] * ph[None, :] * acc
    return 4 * np.pi / case["omega"] * out


def pin_overlap_closed_form(mod):
    case = make_case(1, n_g=120)
    kvec = mod.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    # the closed form takes the matching from its own Cramer solve, not from the oracle
    kn = np.linalg.norm(kvec, axis=1)
    a = np.empty((case["n_types"], case["l_max"] + 1, len(kn)))
    b = np.empty_like(a)
    for t in range(case["n_types"]):
        for l in range(case["l_max"] + 1):
            u, du, ud, dud = case["radial"][t, l]
            x = kn * case["r_mt"][t]
            M = np.array([[u, ud], [du, dud]])
            rhs = np.stack([special.spherical_jn(l, x), kn * special.spherical_jn(l, x, derivative=True)])
            sol = np.linalg.solve(M, rhs)
            a[t, l], b[t, l] = sol
    nrm = case["udot_norm2"]
    ref = _legendre(case, kvec, a, b, lambda t, l, al, bl: np.outer(al, al) + nrm[t, l] * np.outer(bl, bl))
    return _rel(mod.overlap(case, mod.coefficients(case)), ref) < 1e-12


def pin_hamiltonian_diag_blocks(mod):
    case = dict(make_case(1, n_g=100))
    rng = np.random.default_rng(21)
    n_l, l_max = case["n_l"], case["l_max"]
    lL = np.concatenate([[l] * (2 * l + 1) for l in range(l_max + 1)])
    taa, tbb = rng.uniform(-2, 2, (2, case["n_types"], l_max + 1))
    tab = rng.normal(size=(case["n_types"], l_max + 1)) + 1j * rng.normal(size=(case["n_types"], l_max + 1))
    T = np.zeros_like(case["T"])
    for t in range(case["n_types"]):
        T[t, :n_l, :n_l] = np.diag(taa[t][lL])
        T[t, n_l:, n_l:] = np.diag(tbb[t][lL])
        T[t, :n_l, n_l:] = np.diag(tab[t][lL])
        T[t, n_l:, :n_l] = np.diag(np.conj(tab[t][lL]))
    case["T"] = T
    kvec = mod.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    a, b = o.matching(np.linalg.norm(kvec, axis=1), case["r_mt"], case["radial"])  # pinned separately
    ref = _legendre(case, kvec, a, b, lambda t, l, al, bl: taa[t, l] * np.outer(al, al) + tab[t, l] * np.outer(al, bl)
                    + np.conj(tab[t, l]) * np.outer(bl, al) + tbb[t, l] * np.outer(bl, bl))
    return _rel(mod.hamiltonian(case, mod.coefficients(case)), ref) < 1e-12


def pin_covariance(mod):
    case = make_case(1, n_g=100)
    H, S = mod.hs(case)
    d = np.array([0.37, -1.1, 0.52])
    H2, S2 = mod.hs(perturb_positions(case, np.tile(d, (len(case["tau"]), 1))))
    kvec = (case["g"] + case["k_frac"]) @ (2 * np.pi * np.linalg.inv(case["lattice"]).T)
    D = np.exp(1j * kvec @ d)
    return (_rel(H2, np.conj(D)[:, None] * H * D[None, :]) < 1e-12
            and _rel(S2, np.conj(D)[:, None] * S * D[None, :]) < 1e-12)


def pin_tau_fd(mod):
    case = make_case(4, n_g=60)
    Wm, Vm = case["W"], case["V"]
    _, gtau = mod.loss_gradients(case, Wm, Vm)
    h = 1e-6
    worst = 0.0
    for a, c in [(0, 0), (5, 2), (40, 1)]:
        dd = np.zeros_like(case["tau"])
        dd[a, c] = h
        fd = (o.loss(perturb_positions(case, dd), Wm, Vm) - o.loss(perturb_positions(case, -dd), Wm, Vm)) / (2 * h)
        worst = max(worst, abs(fd - gtau[a, c]))
    return worst <= 1e-7 * np.abs(gtau).max()


def pin_gamma(mod):
    """k = 0: the K = 0 column of the coefficients in closed form from the radial data
    (only A_00 = sqrt(4 pi/Omega) udot'/W_0 and B_00 = -sqrt(4 pi/Omega) u'/W_0 nonzero),
    and S_00 = (4 pi/Omega) sum_a (a_0^2 + |udot_0|^2 b_0^2)."""
    case = at_k(make_case(1, n_g=50), np.zeros(3), 123)
    coef = mod.coefficients(case)
    if not np.all(np.isfinite(coef)):
        return False
    pre = np.sqrt(4 * np.pi / case["omega"])
    s00 = 0.0
    for a in range(case["n_atoms"]):
        t = int(case["atom_type"][a])
        u, du, ud, dud = case["radial"][t, 0]
        w = u * dud - ud * du
        a0, b0 = pre * dud / w, -pre * du / w
        if abs(coef[a, 0, 0, 0] - a0) > 1e-14 * abs(a0) or abs(coef[a, 1, 0, 0] - b0) > 1e-14 * abs(b0):
            return False
        if np.abs(coef[a, :, 1:, 0]).max() > 0.0:
            return False
        s00 += a0 * a0 + case["udot_norm2"][t, 0] * b0 * b0
    S = mod.overlap(case, coef)
    return abs(S[0, 0] - s00) <= 1e-13 * s00


PINS = [pin_gamma, pin_plane_wave, pin_matching, pin_overlap_closed_form, pin_hamiltonian_diag_blocks, pin_covariance,
        pin_tau_fd]


def _mutants():
    orig_ang, orig_match, orig_coef = o.angular_factor, o.matching, o.coefficients
    orig_overlap, orig_ham, orig_grad = o.overlap, o.hamiltonian, o.loss_gradients

    def no_conj(kvec, l_max):
        return np.conj(orig_ang(kvec, l_max)) * np.array(
            [(1j ** l) ** 2 for l in range(l_max + 1) for _ in range(2 * l + 1)])[:, None]

    def no_il(kvec, l_max):
        return orig_ang(kvec, l_max) / np.array([1j ** l for l in range(l_max + 1) for _ in range(2 * l + 1)])[:, None]

    def swap_ab(kn, r_mt, radial):
        a, b = orig_match(kn, r_mt, radial)
        return b, a

    def phase_sign(case, tau=None, g=None, k_frac=None):
        t = case["tau"] if tau is None else tau
        return orig_coef(case, tau=-np.asarray(t), g=g, k_frac=k_frac)

    def omega_norm(case, tau=None, g=None, k_frac=None):
        return orig_coef(case, tau=tau, g=g, k_frac=k_frac) / np.sqrt(case["omega"]) ** 0.5

    def no_b_overlap(case, coef):
        c = coef.copy()
        c[:, 1] = 0
        return orig_overlap(case, c)

    def t_transposed(case, coef):
        return orig_ham(dict(case, T=np.transpose(case["T"], (0, 2, 1))), coef)

    def no_zero_guard(kvec, l_max):
        # K_hat = K / |K| taken without the K = 0 rule: NaN angles at K = 0
        kn = np.linalg.norm(kvec, axis=1)
        with np.errstate(invalid="ignore", divide="ignore"):
            theta = np.arccos(kvec[:, 2] / kn)
        phi = np.mod(np.arctan2(kvec[:, 1], kvec[:, 0]), 2 * np.pi)
        return np.stack([(1j ** l) * np.conj(special.sph_harm_y(l, m, theta, phi))
                         for l in range(l_max + 1) for m in range(-l, l + 1)])

    def grad_sign(case, Wm, Vm):
        gT, gtau = orig_grad(case, Wm, Vm)
        return gT, -gtau

    return {"angular without conj": ("angular_factor", no_conj), "angular without i^l": ("angular_factor", no_il),
            "a and b swapped": ("matching", swap_ab), "phase sign flipped": ("coefficients", phase_sign),
            "1/sqrt(Omega) squared": ("coefficients", omega_norm), "B term dropped from S": ("overlap", no_b_overlap),
            "T transposed in H": ("hamiltonian", t_transposed), "tau gradient sign": ("loss_gradients", grad_sign),
            "no K = 0 rule for the angles": ("angular_factor", no_zero_guard)}


def test_unmutated_oracle_passes_every_pin():
    for pin in PINS:
        assert pin(o), pin.__name__


@pytest.mark.parametrize("name", sorted(_mutants()))
def test_each_mutation_fails_a_pin(name, monkeypatch):
    attr, fn = _mutants()[name]
    monkeypatch.setattr(o, attr, fn)
    failed = [pin.__name__ for pin in PINS if not pin(o)]
    assert failed, "mutation '%s' passed every pin" % name
