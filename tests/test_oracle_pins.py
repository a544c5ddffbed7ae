"""Pins of the oracle against facts the mathematics fixes (no GPU).

Each test checks the oracle against something other than itself: closed-form
special functions, the plane wave the muffin-tin expansion must reproduce on
the sphere (Sec. 2.1, Eq. 2), the Legendre addition theorem (which gives S,
and H for m-independent diagonal T blocks, in closed form), brute-force
summation of Eq. 5, the paper's own evaluation order (Alg. 3), the matrix
properties stated in Sec. 2.2, and translation invariance/covariance.
"""
import numpy as np
import pytest
from scipy import special

from flapw_cells import at_k, make_case, perturb_positions
from oracle import hs_oracle as o


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def case0():
    return make_case(0)


@pytest.fixture(scope="module")
def hs0(case0):
    return o.hs(case0)


def small_case(index=1, n_g=160):
    return make_case(index, n_g=n_g)


# ---- special functions and matching --------------------------------------------------

def _j_closed(l, x):
    s, c = np.sin(x), np.cos(x)
    if l == 0:
        return s / x, (x * c - s) / x ** 2
    if l == 1:
        return s / x ** 2 - c / x, (x ** 2 * s + 2 * x * c - 2 * s) / x ** 3
    if l == 2:
        j = (3 / x ** 3 - 1 / x) * s - 3 * c / x ** 2
        dj = (-9 / x ** 4 + 1 / x ** 2) * s + (3 / x ** 3 - 1 / x) * c + 6 * c / x ** 3 + 3 * s / x ** 2
        return j, dj
    raise ValueError


def test_matching_reproduces_closed_form_bessel():
    """a_l u + b_l udot = j_l(x) and a_l u' + b_l udot' = |K| j_l'(x), with j_0..j_2
    written from sin/cos (value and slope continuity at R_MT, Sec. 2.1)."""
    rng = np.random.default_rng(3)
    kn = rng.uniform(0.3, 4.0, 50)
    r_mt = np.array([1.7])
    radial = rng.uniform(0.5, 1.5, (1, 3, 4))
    a, b = o.matching(kn, r_mt, radial)
    x = kn * r_mt[0]
    for l in range(3):
        j, dj = _j_closed(l, x)
        u, du, ud, dud = radial[0, l]
        np.testing.assert_allclose(a[0, l] * u + b[0, l] * ud, j, rtol=0, atol=1e-12)
        np.testing.assert_allclose(a[0, l] * du + b[0, l] * dud, kn * dj, rtol=0, atol=1e-12)


def test_matching_small_argument_limit():
    """For x -> 0, j_l(x) ~ x^l/(2l+1)!!: check the value condition at x = 1e-3."""
    kn = np.array([1e-3])
    radial = np.tile(np.array([1.0, 0.3, 0.7, 1.2]), (1, 11, 1))
    a, b = o.matching(kn, np.array([1.0]), radial)
    for l in range(11):
        dfact = np.prod(np.arange(1, 2 * l + 2, 2, dtype=float))
        approx = kn[0] ** l / dfact * (1 - kn[0] ** 2 / (2 * (2 * l + 3)))
        val = a[0, l, 0] * 1.0 + b[0, l, 0] * 0.7
        assert abs(val - approx) <= 1e-9 * abs(approx)


def test_angular_factor_low_order_closed_forms():
    """i^l conj(Y_lm) for l <= 2 against the Cartesian forms of the complex
    harmonics with Condon-Shortley phase."""
    rng = np.random.default_rng(5)
    v = rng.normal(size=(40, 3))
    ang = o.angular_factor(v, 2)
    r = np.linalg.norm(v, axis=1)
    x, y, z = (v / r[:, None]).T
    pi = np.pi
    Y = {
        (0, 0): np.full_like(x, np.sqrt(1 / (4 * pi))) + 0j,
        (1, 0): np.sqrt(3 / (4 * pi)) * z + 0j,
        (1, 1): -np.sqrt(3 / (8 * pi)) * (x + 1j * y),
        (1, -1): np.sqrt(3 / (8 * pi)) * (x - 1j * y),
        (2, 0): np.sqrt(5 / (16 * pi)) * (3 * z ** 2 - 1) + 0j,
        (2, 1): -np.sqrt(15 / (8 * pi)) * z * (x + 1j * y),
        (2, -1): np.sqrt(15 / (8 * pi)) * z * (x - 1j * y),
        (2, 2): np.sqrt(15 / (32 * pi)) * (x + 1j * y) ** 2,
        (2, -2): np.sqrt(15 / (32 * pi)) * (x - 1j * y) ** 2,
    }
    for (l, m), ylm in Y.items():
        np.testing.assert_allclose(ang[o.lm_index(l, m)], (1j ** l) * np.conj(ylm), rtol=0, atol=1e-14)


def test_angular_factor_zero_vector_is_z_axis():
    ang = o.angular_factor(np.zeros((1, 3)), 3)
    ref = o.angular_factor(np.array([[0.0, 0.0, 1.0]]), 3)
    np.testing.assert_allclose(ang, ref, atol=0)


def test_addition_theorem():
    """sum_m Y*_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b) for l <= 12."""
    rng = np.random.default_rng(11)
    u = rng.normal(size=(30, 3))
    w = rng.normal(size=(30, 3))
    au = o.angular_factor(u, 12)
    aw = o.angular_factor(w, 12)
    cosg = np.einsum("ij,ij->i", u, w) / np.linalg.norm(u, axis=1) / np.linalg.norm(w, axis=1)
    for l in range(13):
        sl = slice(l * l, (l + 1) ** 2)
        # i^l conj(Y) on both sides: conj(au) * aw = Y(u) conj(Y(w))
        lhs = np.sum(np.conj(au[sl]) * aw[sl], axis=0)
        np.testing.assert_allclose(lhs, (2 * l + 1) / (4 * np.pi) * special.eval_legendre(l, cosg),
                                   rtol=0, atol=1e-13)


# ---- coefficients: the muffin-tin expansion equals the plane wave on the sphere ---------

def test_boundary_continuity_plane_wave():
    """sum_L [A_L u_l(R) + B_L udot_l(R)] Y_L(r_hat) = e^{iK.(tau + R r_hat)} / sqrt(Omega)
    on the sphere of atom a (Eq. 2 continuous with the interstitial plane wave).
    l_max = 14 and |K| R <= 1 make the truncated Rayleigh series exact to ~1e-14."""
    base = make_case(0, n_g=256)
    l_max = 14
    case = dict(base)
    case["l_max"] = l_max
    rng = np.random.default_rng(7)
    case["radial"] = rng.uniform(0.5, 1.5, (1, l_max + 1, 4))
    # keep only G with |K| R <= 1
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    keep = np.linalg.norm(kvec, axis=1) * case["r_mt"][0] <= 1.0
    g = case["g"][keep]
    assert len(g) >= 3
    coef = o.coefficients(case, g=g)
    kvec = kvec[keep]
    R = case["r_mt"][0]
    pts = rng.normal(size=(25, 3))
    pts /= np.linalg.norm(pts, axis=1)[:, None]
    theta = np.arccos(pts[:, 2])
    phi = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi)
    Ypts = np.stack([special.sph_harm_y(l, m, theta, phi) for l in range(l_max + 1) for m in range(-l, l + 1)])
    u = np.concatenate([[case["radial"][0, l, 0]] * (2 * l + 1) for l in range(l_max + 1)])
    ud = np.concatenate([[case["radial"][0, l, 2]] * (2 * l + 1) for l in range(l_max + 1)])
    for a in range(len(case["tau"])):
        val = (coef[a, 0] * u[:, None] + coef[a, 1] * ud[:, None]).T @ Ypts  # [G, point]
        r = case["tau"][a][None, :] + R * pts
        pw = np.exp(1j * kvec @ r.T) / np.sqrt(case["omega"])
        np.testing.assert_allclose(val, pw, rtol=0, atol=1e-13)


# ---- k on a lattice point: the basis holds K = k + G = 0 (Sec. 2.1) ---------------------
# At K = 0 only l = 0 survives: j_0(0) = 1, j_l(0) = 0 for l >= 1 and |K| j_l'(0) = 0, so
# a_0 = udot'/W_0, b_0 = -u'/W_0 (W_0 = u udot' - udot u'), every other a_l, b_l is 0, the
# phase is 1 and Y_00 = 1/sqrt(4 pi) whatever direction K_hat is given.

def gamma_case(index=1, n_g=123):
    """Workload `index` moved to k = 0 with a closed-shell basis (G = 0 first)."""
    case = at_k(make_case(index, n_g=50), np.zeros(3), n_g)
    assert np.all(case["g"][0] == 0)
    return case


def _w0(radial_tl):
    u, du, ud, dud = radial_tl
    return u * dud - ud * du


def test_matching_at_zero_argument():
    """x = 0 in the matching: a_0 = udot'/W_0, b_0 = -u'/W_0 and a_l = b_l = 0 for l >= 1
    (the value and slope of the plane wave at K = 0 are 1 and 0)."""
    radial = np.random.default_rng(31).uniform(0.5, 1.5, (2, 13, 4))
    a, b = o.matching(np.zeros(3), np.array([1.2, 2.3]), radial)
    for t in range(2):
        u, du, ud, dud = radial[t, 0]
        np.testing.assert_allclose(a[t, 0], dud / _w0(radial[t, 0]), rtol=1e-15, atol=0)
        np.testing.assert_allclose(b[t, 0], -du / _w0(radial[t, 0]), rtol=1e-15, atol=0)
        assert np.all(a[t, 1:] == 0.0) and np.all(b[t, 1:] == 0.0)


def test_gamma_coefficients_of_g0_closed_form():
    """The G = 0 column at k = 0: A_00 = sqrt(4 pi/Omega) a_0 and B_00 = sqrt(4 pi/Omega) b_0
    for every atom (phase 1, whatever its position), every other (l, m) exactly 0; the
    values come from the radial data alone."""
    case = gamma_case(1, 123)
    coef = o.coefficients(case)
    pre = np.sqrt(4 * np.pi / case["omega"])
    for a in range(case["n_atoms"]):
        r = case["radial"][int(case["atom_type"][a]), 0]
        u, du, ud, dud = r
        np.testing.assert_allclose(coef[a, 0, 0, 0], pre * dud / _w0(r), rtol=1e-14, atol=0)
        np.testing.assert_allclose(coef[a, 1, 0, 0], -pre * du / _w0(r), rtol=1e-14, atol=0)
        assert np.all(coef[a, :, 1:, 0] == 0.0)


def test_gamma_boundary_continuity_plane_wave():
    """The muffin-tin expansion equals the plane wave on the sphere at k = 0, the K = 0
    column (constant 1/sqrt(Omega)) included; |K| R <= 1 with l_max 14 as above."""
    case = gamma_case(0, 123)
    l_max = 14
    case = dict(case, l_max=l_max)
    rng = np.random.default_rng(17)
    case["radial"] = rng.uniform(0.5, 1.5, (1, l_max + 1, 4))
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    keep = np.linalg.norm(kvec, axis=1) * case["r_mt"][0] <= 1.0
    assert keep[0] and keep.sum() >= 7
    coef = o.coefficients(case, g=case["g"][keep])
    kvec = kvec[keep]
    R = case["r_mt"][0]
    pts = rng.normal(size=(25, 3))
    pts /= np.linalg.norm(pts, axis=1)[:, None]
    theta = np.arccos(pts[:, 2])
    phi = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi)
    Ypts = np.stack([special.sph_harm_y(l, m, theta, phi) for l in range(l_max + 1) for m in range(-l, l + 1)])
    u = np.concatenate([[case["radial"][0, l, 0]] * (2 * l + 1) for l in range(l_max + 1)])
    ud = np.concatenate([[case["radial"][0, l, 2]] * (2 * l + 1) for l in range(l_max + 1)])
    for a in range(len(case["tau"])):
        val = (coef[a, 0] * u[:, None] + coef[a, 1] * ud[:, None]).T @ Ypts
        pw = np.exp(1j * kvec @ (case["tau"][a][None, :] + R * pts).T) / np.sqrt(case["omega"])
        np.testing.assert_allclose(val, pw, rtol=0, atol=1e-13)
        np.testing.assert_allclose(val[0], 1.0 / np.sqrt(case["omega"]), rtol=0, atol=1e-15)


def test_gamma_overlap_and_hamiltonian_closed_form():
    """At k = 0: the whole S by the Legendre closed form (only l = 0 enters the K = 0 row
    and column, so the K_hat convention cannot matter), the row of S and of H at G' = 0 in
    closed form from the radial data, the phases and T's (l = 0) entries alone:
      S_0G = (4 pi/Omega) sum_a e^{iK_G.tau_a} [a_0(0) a_0(K_G) + |udot_0|^2 b_0(0) b_0(K_G)],
      H_0G = (4 pi/Omega) sum_a e^{iK_G.tau_a} [a_0(0), b_0(0)] T_t[(A|B,00), (A|B,L)] [A|B coefficients],
    and S_00, H_00 from the radial values only."""
    case = gamma_case(1, 123)
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    assert np.linalg.norm(kvec[0]) == 0.0
    coef = o.coefficients(case)
    H, S = o.hamiltonian(case, coef), o.overlap(case, coef)
    # Legendre form of S with the matching by an independent Cramer solve at every G
    kn = np.linalg.norm(kvec, axis=1)
    a = np.empty((case["n_types"], case["l_max"] + 1, len(kn)))
    b = np.empty_like(a)
    for t in range(case["n_types"]):
        for l in range(case["l_max"] + 1):
            u, du, ud, dud = case["radial"][t, l]
            x = kn * case["r_mt"][t]
            rhs = np.stack([special.spherical_jn(l, x), kn * special.spherical_jn(l, x, derivative=True)])
            a[t, l], b[t, l] = np.linalg.solve(np.array([[u, ud], [du, dud]]), rhs)
    nrm = case["udot_norm2"]
    ref = _legendre_form(case, a, b, kvec, lambda t, l, al, bl: np.outer(al, al) + nrm[t, l] * np.outer(bl, bl))
    assert rel(S, ref) < 1e-13
    # row G' = 0 of S and H, and the (0, 0) entries
    pre2 = 4 * np.pi / case["omega"]
    n_l = case["n_l"]
    s_row = np.zeros(case["n_g"], dtype=np.complex128)
    h_row = np.zeros(case["n_g"], dtype=np.complex128)
    s00 = h00 = 0.0
    for at in range(case["n_atoms"]):
        t = int(case["atom_type"][at])
        r = case["radial"][t, 0]
        a0, b0 = r[3] / _w0(r), -r[1] / _w0(r)
        ph = np.exp(1j * (kvec @ case["tau"][at]))
        s_row += pre2 * ph * (a0 * a[t, 0] + nrm[t, 0] * b0 * b[t, 0])
        Tt = case["T"][t]
        Wa = coef[at].reshape(2 * n_l, -1)
        h_row += np.sqrt(pre2) * (a0 * Tt[0] + b0 * Tt[n_l]) @ Wa  # conj of a real row
        s00 += pre2 * (a0 * a0 + nrm[t, 0] * b0 * b0)
        h00 += pre2 * (a0 * a0 * Tt[0, 0].real + 2 * a0 * b0 * Tt[0, n_l].real + b0 * b0 * Tt[n_l, n_l].real)
    assert rel(S[0], s_row) < 1e-13 and rel(H[0], h_row) < 1e-13
    assert abs(S[0, 0] - s00) <= 1e-14 * abs(s00) and abs(H[0, 0] - h00) <= 1e-13 * abs(h00)


def test_gamma_hermitian_and_translation_invariant():
    case = gamma_case(0, 57)
    H, S = o.hs(case)
    assert rel(H, H.conj().T) < 1e-15 and rel(S, S.conj().T) < 1e-15
    shift = np.tile(case["lattice"][0] - 2 * case["lattice"][2], (case["n_atoms"], 1))
    H2, S2 = o.hs(perturb_positions(case, shift))
    assert rel(H2, H) < 1e-13 and rel(S2, S) < 1e-13


# ---- closed forms of S and H ---------------------------------------------------------

def _legendre_form(case, coef_a, coef_b, kvec, weights):
    """(4 pi / Omega) sum_a e^{i(K_G - K_G').tau_a} sum_l (2l+1) P_l(K_hat'.K_hat) w_l(G', G)."""
    n = len(kvec)
    kn = np.linalg.norm(kvec, axis=1)
    khat = np.where(kn[:, None] > 1e-12, kvec / np.where(kn > 1e-12, kn, 1.0)[:, None], [0, 0, 1.0])
    cosg = np.clip(khat @ khat.T, -1.0, 1.0)
    out = np.zeros((n, n), dtype=np.complex128)
    for a, tau in enumerate(case["tau"]):
        t = int(case["atom_type"][a])
        ph = np.exp(1j * (kvec @ tau))
        acc = np.zeros((n, n), dtype=np.complex128)
        for l in range(case["l_max"] + 1):
            acc += (2 * l + 1) * special.eval_legendre(l, cosg) * weights(t, l, coef_a[t, l], coef_b[t, l])
        out += np.conj(ph)[:, None] * ph[None, :] * acc
    return 4 * np.pi / case["omega"] * out


def test_overlap_closed_form_any_positions():
    case = small_case(1, 200)
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    a, b = o.matching(np.linalg.norm(kvec, axis=1), case["r_mt"], case["radial"])
    nrm = case["udot_norm2"]
    ref = _legendre_form(case, a, b, kvec,
                         lambda t, l, al, bl: np.outer(al, al) + nrm[t, l] * np.outer(bl, bl))
    S = o.overlap(case, o.coefficients(case))
    assert rel(S, ref) < 1e-13


def test_hamiltonian_closed_form_diagonal_blocks():
    """T blocks diagonal in L and depending on l only (T^AB complex):
    H = (4 pi/Omega) sum_a phases sum_l (2l+1) P_l [taa a'a + tab a'b + conj(tab) b'a + tbb b'b]."""
    case = dict(small_case(1, 150))
    rng = np.random.default_rng(21)
    n_l, l_max = case["n_l"], case["l_max"]
    l_of_L = np.concatenate([[l] * (2 * l + 1) for l in range(l_max + 1)])
    taa = rng.uniform(-2, 2, (case["n_types"], l_max + 1))
    tbb = rng.uniform(-2, 2, (case["n_types"], l_max + 1))
    tab = rng.normal(size=(case["n_types"], l_max + 1)) + 1j * rng.normal(size=(case["n_types"], l_max + 1))
    T = np.zeros_like(case["T"])
    for t in range(case["n_types"]):
        T[t, :n_l, :n_l] = np.diag(taa[t][l_of_L])
        T[t, n_l:, n_l:] = np.diag(tbb[t][l_of_L])
        T[t, :n_l, n_l:] = np.diag(tab[t][l_of_L])
        T[t, n_l:, :n_l] = np.diag(np.conj(tab[t][l_of_L]))
    case["T"] = T
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    a, b = o.matching(np.linalg.norm(kvec, axis=1), case["r_mt"], case["radial"])

    def w(t, l, al, bl):
        return (taa[t, l] * np.outer(al, al) + tab[t, l] * np.outer(al, bl)
                + np.conj(tab[t, l]) * np.outer(bl, al) + tbb[t, l] * np.outer(bl, bl))

    ref = _legendre_form(case, a, b, kvec, w)
    H = o.hamiltonian(case, o.coefficients(case))
    assert rel(H, ref) < 1e-13


def test_hamiltonian_type_hadamard_identity():
    """H = sum_t (W0_t^H T_t W0_t) o (E_t^H E_t), W0 the coefficients at tau = 0 and
    E_t[a, G] = e^{iK_G.tau_a} over the atoms of type t (T shared per type)."""
    case = small_case(1, 180)
    H = o.hamiltonian(case, o.coefficients(case))
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    c0 = o.coefficients(case, tau=np.zeros_like(case["tau"]))
    ref = np.zeros_like(H)
    for t in range(case["n_types"]):
        atoms = np.nonzero(case["atom_type"] == t)[0]
        W0 = c0[atoms[0]].reshape(2 * case["n_l"], -1)
        M = W0.conj().T @ case["T"][t] @ W0
        E = np.exp(1j * case["tau"][atoms] @ kvec.T)
        ref += M * (E.conj().T @ E)
    assert rel(H, ref) < 1e-13


def test_hamiltonian_bruteforce_eq5():
    case = make_case(0, n_g=10)
    coef = o.coefficients(case)
    np.testing.assert_allclose(o.hamiltonian(case, coef), o.hamiltonian_bruteforce(case, coef),
                               rtol=0, atol=1e-12)


def test_paper_evaluation_order_alg3(case0, hs0):
    """The refined HSDLA order (Alg. 3): S = A^H A + (U B)^H (U B);
    Z = T^BA A + 1/2 T^BB B stacked; H = Z^H B + B^H Z (zher2k); X = T^AA A;
    H += A^H X (zherkx).  Same result as the fused evaluation."""
    case = case0
    coef = o.coefficients(case)
    n_at, _, n_l, n = coef.shape
    l_of_L = np.concatenate([[l] * (2 * l + 1) for l in range(case["l_max"] + 1)])
    As, Bs, Xs, Zs, UBs = [], [], [], [], []
    for a in range(n_at):
        Tt = case["T"][int(case["atom_type"][a])]
        A, B = coef[a, 0], coef[a, 1]
        U = np.sqrt(case["udot_norm2"][int(case["atom_type"][a])][l_of_L])
        TAA, TAB, TBA, TBB = Tt[:n_l, :n_l], Tt[:n_l, n_l:], Tt[n_l:, :n_l], Tt[n_l:, n_l:]
        np.testing.assert_allclose(TBA, TAB.conj().T, atol=0)
        Zs.append(TBA @ A + 0.5 * TBB @ B)
        Xs.append(TAA @ A)
        As.append(A)
        Bs.append(B)
        UBs.append(U[:, None] * B)
    A, B, X, Z, UB = (np.concatenate(v) for v in (As, Bs, Xs, Zs, UBs))
    S = A.conj().T @ A + UB.conj().T @ UB
    H = Z.conj().T @ B + B.conj().T @ Z + A.conj().T @ X
    H_ref, S_ref = hs0
    assert rel(S, S_ref) < 1e-14
    assert rel(H, H_ref) < 1e-14


# ---- matrix properties (Sec. 2.2) and translations ---------------------------------------

def test_hermitian_and_psd(hs0):
    H, S = hs0
    assert np.abs(H - H.conj().T).max() <= 1e-13 * np.abs(H).max()
    assert np.abs(S - S.conj().T).max() <= 1e-13 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.conj().T))
    assert ev.min() >= -1e-13 * ev.max()
    evh = np.linalg.eigvalsh(0.5 * (H + H.conj().T))
    assert evh.min() < 0 < evh.max()  # H indefinite


def test_lattice_translation_invariance():
    case = small_case(1, 150)
    H, S = o.hs(case)
    shift = np.zeros_like(case["tau"])
    shift[:] = case["lattice"][0] - 2 * case["lattice"][2]
    H2, S2 = o.hs(perturb_positions(case, shift))
    assert rel(H2, H) < 1e-12 and rel(S2, S) < 1e-12
    one = np.zeros_like(case["tau"])
    one[3] = case["lattice"][1]
    H3, S3 = o.hs(perturb_positions(case, one))
    assert rel(H3, H) < 1e-12 and rel(S3, S) < 1e-12


def test_general_translation_covariance():
    """Moving every atom by d multiplies each coefficient column by e^{iK_G.d}:
    H(tau + d) = D^H H D with D = diag(e^{iK_G.d})."""
    case = small_case(1, 150)
    H, S = o.hs(case)
    d = np.array([0.37, -1.1, 0.52])
    H2, S2 = o.hs(perturb_positions(case, np.tile(d, (len(case["tau"]), 1))))
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    D = np.exp(1j * kvec @ d)
    assert rel(H2, np.conj(D)[:, None] * H * D[None, :]) < 1e-12
    assert rel(S2, np.conj(D)[:, None] * S * D[None, :]) < 1e-12


def test_hs_entries_match_full(case0, hs0):
    rng = np.random.default_rng(1)
    rows = rng.integers(0, case0["n_g"], 40)
    cols = rng.integers(0, case0["n_g"], 40)
    h, s = o.hs_entries(case0, rows, cols)
    np.testing.assert_allclose(h, hs0[0][rows, cols], rtol=0, atol=1e-12)
    np.testing.assert_allclose(s, hs0[1][rows, cols], rtol=0, atol=1e-12)


# ---- gradients ----------------------------------------------------------------------

@pytest.fixture(scope="module")
def grad_case():
    case = make_case(4, n_g=120)
    return case


def test_gradient_tau_central_difference(grad_case):
    case = grad_case
    Wm, Vm = case["W"], case["V"]
    gT, gtau = o.loss_gradients(case, Wm, Vm)
    h = 1e-6
    rng = np.random.default_rng(2)
    picks = [(int(a), int(c)) for a, c in zip(rng.integers(0, case["n_atoms"], 10), rng.integers(0, 3, 10))]
    for a, c in picks:
        d = np.zeros_like(case["tau"])
        d[a, c] = h
        lp = o.loss(perturb_positions(case, d), Wm, Vm)
        lm = o.loss(perturb_positions(case, -d), Wm, Vm)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gtau[a, c]) <= 1e-7 * np.abs(gtau).max() + 1e-12


def test_gradient_T_directional(grad_case):
    """L is linear in T: a central difference along a Hermitian direction is exact."""
    case = dict(grad_case)
    Wm, Vm = case["W"], case["V"]
    gT, _ = o.loss_gradients(case, Wm, Vm)
    rng = np.random.default_rng(4)
    m = case["T"].shape[1]
    for _ in range(3):
        D = rng.normal(size=case["T"].shape) + 1j * rng.normal(size=case["T"].shape)
        D = D + np.conj(np.transpose(D, (0, 2, 1)))
        h = 1e-7
        cp = dict(case, T=case["T"] + h * D)
        cm = dict(case, T=case["T"] - h * D)
        fd = (o.loss(cp, Wm, Vm) - o.loss(cm, Wm, Vm)) / (2 * h)
        pred = float(np.real(np.sum(np.conj(gT) * D)))
        assert abs(fd - pred) <= 1e-7 * abs(pred) + 1e-9
    assert m == 2 * case["n_l"]


def test_gradient_euler_identity(grad_case):
    """L_H = Re tr(W H) is linear in T, so sum_t Re <grad_T, T> = L_H (V = 0)."""
    case = grad_case
    Wm = case["W"]
    Vm = np.zeros_like(Wm)
    gT, _ = o.loss_gradients(case, Wm, Vm)
    lh = o.loss(case, Wm, Vm)
    assert abs(float(np.real(np.sum(np.conj(gT) * case["T"]))) - lh) <= 1e-12 * abs(lh)


def test_gradient_translation_sum_rule(grad_case):
    """sum_a grad_tau_a = Re sum_{GG'} i (K_G - K_G') [W_{GG'} H_{G'G} + V_{GG'} S_{G'G}]."""
    case = grad_case
    Wm, Vm = case["W"], case["V"]
    _, gtau = o.loss_gradients(case, Wm, Vm)
    H, S = o.hs(case)
    kvec = o.k_plus_g(case["lattice"], case["k_frac"], case["g"])
    M = Wm.T * H + Vm.T * S
    for c in range(3):
        dk = kvec[None, :, c] - kvec[:, None, c]
        total = float(np.real(np.sum(1j * dk * M)))
        assert abs(gtau[:, c].sum() - total) <= 1e-12 * np.abs(gtau).max()


# ---- flop accounting against the paper's Table 1 and Alg. 3 annotations ---------------------

def test_flops_vs_paper_alg3_counts():
    """The paper's Alg. 3 annotations add to 20 N_A N_L N_G^2 + 24 N_A N_L^2 N_G (plus
    scaling); the fused Hermitian form needs 16 N_A N_L N_G (N_G+1) + 32 N_A N_L^2 N_G.
    The sizes are the paper's Table 1 (tests/golden/table1_sizes.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_sizes.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 12
    for name, n_a, n_l, kmax, n_g in rows:
        n_a, n_l, n_g = int(n_a), int(n_l), int(n_g)
        lmax = int(round(np.sqrt(n_l))) - 1
        assert (lmax + 1) ** 2 == n_l  # N_L = (l_max + 1)^2 in every workload
        paper = 20.0 * n_a * n_l * n_g ** 2 + 24.0 * n_a * n_l ** 2 * n_g
        ours = o.flops_forward(n_a, n_l, n_g)
        assert 1.2 < paper / ours < 1.26


def test_inversion_symmetric_cell_gives_real_h_and_s():
    """With the atoms in inversion pairs about the origin and T invariant under
    time reversal and site inversion, each pair's contribution is twice the
    real part of one member's, so H and S are real symmetric (the real case of
    Sec. 2.1).  Breaking either symmetry brings back an imaginary part."""
    from flapw_cells import make_case
    case = make_case(5, n_g=300)
    H, S = o.hs(case)
    assert np.linalg.norm(H.imag) <= 1e-13 * np.linalg.norm(H)
    assert np.linalg.norm(S.imag) <= 1e-13 * np.linalg.norm(S)
    # a general Hermitian T on the same positions: H complex, S (T-free) still real
    rng = np.random.default_rng(3)
    m = 2 * case["n_l"]
    Z = rng.normal(size=(case["n_types"], m, m)) + 1j * rng.normal(size=(case["n_types"], m, m))
    H2, _ = o.hs(dict(case, T=0.05 * (Z + np.conj(np.transpose(Z, (0, 2, 1))))))
    assert np.linalg.norm(H2.imag) > 1e-3 * np.linalg.norm(H2)
    # move one atom off its pair position: S picks up an imaginary part
    tau = case["tau"].copy()
    tau[0] += np.array([0.31, -0.2, 0.05])
    _, S3 = o.hs(dict(case, tau=tau))
    assert np.linalg.norm(S3.imag) > 1e-3 * np.linalg.norm(S3)


def test_generalized_eigenvalues_by_an_independent_reduction():
    """The pencil's eigenvalues equal those of the standard problem
    L^{-1} H L^{-H} (S = L L^H, Cholesky by hand-written forward substitution
    in numpy, eigenvalues by numpy's eigvalsh); on the bench cell at N_G = 400
    the muffin-tin S is positive definite (2 N_at N_L = 30976 > N_G)."""
    from flapw_cells import make_case
    case = make_case(2, n_g=400)
    H, S = o.hs(case)
    w = o.generalized_eigenvalues(H, S)
    L = np.linalg.cholesky(S)
    n = len(S)
    Linv = np.zeros_like(S)
    eye = np.eye(n, dtype=S.dtype)
    for i in range(n):  # forward substitution, row by row
        Linv[i] = (eye[i] - L[i, :i] @ Linv[:i]) / L[i, i]
    ref = np.linalg.eigvalsh(Linv @ H @ Linv.conj().T)
    assert np.abs(w - ref).max() <= 1e-9 * np.abs(ref).max()
    # the pencil is not the standard problem: S != I changes the spectrum
    assert np.abs(np.linalg.eigvalsh(H) - ref).max() > 1e-3 * np.abs(ref).max()
