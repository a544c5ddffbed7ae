"""Oracle for the muffin-tin Hamiltonian and overlap matrices (FLAPW, HSDLA).

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain CPU evaluation that
the GPU library is checked against.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the library never does,
and it shares no code, tables or constants with the library.  Everything is
complex128 / float64.

What it computes, in the paper's notation (Sec. 2, Eqs. 2-7):

* the LAPW basis of one k-point is the plane waves e^{i(k+G).r} with
  |k+G| <= K_max (Sec. 2.1); inside muffin-tin sphere a of radius R_MT the
  same function is  sum_{lm} [A^{a,G}_{lm} u_l(r) + B^{a,G}_{lm} udot_l(r)]
  Y_lm(r_hat)  (Eq. 2), with A and B fixed by continuity of value and slope
  at the sphere boundary (Sec. 2.1).  The paper gives no formula for them;
  the standard LAPW matching is used: with K = k+G, x = |K| R_MT and the
  Rayleigh expansion e^{iK.r} = 4 pi sum_lm i^l j_l(|K| r) conj(Y_lm(K_hat))
  Y_lm(r_hat),
      a_l u + b_l udot   = j_l(x),   a_l u' + b_l udot' = |K| j_l'(x),
      A^{a,G}_{lm} = (4 pi / sqrt(Omega)) e^{iK.tau_a} i^l conj(Y_lm(K_hat)) a_l,
  and B the same with b_l.
* S (Eq. 4, matrix form Eq. 7):  S_{G'G} = sum_a sum_L conj(A^{G'}) A^{G}
  + ||udot_l||^2 conj(B^{G'}) B^{G}.
* H (Eq. 5, matrix form Eq. 6):  H = sum_a W_a^H T_a W_a with
  W_a = [A_a; B_a] and T_a = [[T^AA, T^AB], [T^BA, T^BB]], T^BA = (T^AB)^H.

The index a runs over atoms; T and ||udot||^2 depend only on the atom's type.
"""
from __future__ import annotations

import numpy as np
from scipy import special

FOUR_PI = 4.0 * np.pi


def lm_index(l: int, m: int) -> int:
    """Compound index L of (l, m): l^2 + l + m, m from -l to l."""
    return l * l + l + m


def reciprocal_vectors(lattice: np.ndarray) -> np.ndarray:
    """Rows b_j with a_i . b_j = 2 pi delta_ij (lattice rows are a_i)."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def k_plus_g(lattice, k_frac, g) -> np.ndarray:
    """Cartesian K_G = (G + k) in the reciprocal basis, one row per G (Sec. 2.1)."""
    return (np.asarray(g, dtype=np.float64) + np.asarray(k_frac, dtype=np.float64)) @ reciprocal_vectors(lattice)


def direction_angles(kvec: np.ndarray):
    """Polar and azimuthal angle of K_hat; K = 0 takes the z axis."""
    kn = np.linalg.norm(kvec, axis=1)
    zero = kn < 1e-12
    cos_t = np.where(zero, 1.0, kvec[:, 2] / np.where(zero, 1.0, kn))
    theta = np.arccos(np.clip(cos_t, -1.0, 1.0))
    phi = np.where(zero, 0.0, np.mod(np.arctan2(kvec[:, 1], kvec[:, 0]), 2.0 * np.pi))
    return kn, theta, phi


def angular_factor(kvec: np.ndarray, l_max: int) -> np.ndarray:
    """i^l conj(Y_lm(K_hat)) for every L and G: complex [N_L, n].  Y_lm is the
    complex orthonormal harmonic with the Condon-Shortley phase."""
    _, theta, phi = direction_angles(kvec)
    out = np.empty(((l_max + 1) ** 2, len(kvec)), dtype=np.complex128)
    for l in range(l_max + 1):
        for m in range(-l, l + 1):
            out[lm_index(l, m)] = (1j ** l) * np.conj(special.sph_harm_y(l, m, theta, phi))
    return out


def matching(kn: np.ndarray, r_mt: np.ndarray, radial: np.ndarray):
    """a_l and b_l per (type, l, G) from value and slope continuity at R_MT
    (Sec. 2.1): a u + b udot = j_l(x), a u' + b udot' = |K| j_l'(x), x = |K| R.
    radial[t, l] = (u, u', udot, udot') at R_MT.  Returns (a, b), [n_types, l_max+1, n]."""
    n_types, lp1, _ = radial.shape
    a = np.empty((n_types, lp1, len(kn)))
    b = np.empty_like(a)
    for t in range(n_types):
        x = kn * r_mt[t]
        for l in range(lp1):
            jl = special.spherical_jn(l, x)
            djl = kn * special.spherical_jn(l, x, derivative=True)
            u, du, ud, dud = radial[t, l]
            # Cramer's rule on [[u, ud], [du, dud]] [a, b]^T = [jl, djl]^T
            det = u * dud - ud * du
            a[t, l] = (jl * dud - ud * djl) / det
            b[t, l] = (u * djl - du * jl) / det
    return a, b


def coefficients(case: dict, tau=None, g=None, k_frac=None) -> np.ndarray:
    """The stacked matching coefficients  W[a, 0, L, G] = A^{a,G}_L  and
    W[a, 1, L, G] = B^{a,G}_L  (Eq. 2 with the matching above).  Optional
    arguments replace the case's positions, G list or k-point."""
    tau = case["tau"] if tau is None else np.asarray(tau)
    g = case["g"] if g is None else np.asarray(g)
    k_frac = case["k_frac"] if k_frac is None else np.asarray(k_frac)
    l_max = int(case["l_max"])
    kvec = k_plus_g(case["lattice"], k_frac, g)
    kn = np.linalg.norm(kvec, axis=1)
    ang = angular_factor(kvec, l_max)
    a, b = matching(kn, case["r_mt"], case["radial"])
    l_of_L = np.concatenate([[l] * (2 * l + 1) for l in range(l_max + 1)])
    pre = FOUR_PI / np.sqrt(case["omega"])
    n_at = len(tau)
    out = np.empty((n_at, 2, len(l_of_L), len(g)), dtype=np.complex128)
    for alpha in range(n_at):
        t = int(case["atom_type"][alpha])
        phase = np.exp(1j * (kvec @ tau[alpha]))
        out[alpha, 0] = pre * phase[None, :] * ang * a[t][l_of_L]
        out[alpha, 1] = pre * phase[None, :] * ang * b[t][l_of_L]
    return out


def overlap(case: dict, coef: np.ndarray) -> np.ndarray:
    """S of Eq. 4: the sum over atoms a and (l, m) of conj(A^{G'}) A^{G} +
    ||udot_l||^2 conj(B^{G'}) B^{G}, written as one product over the stacked
    index (a, L) (Eq. 7)."""
    n_at, _, n_l, n = coef.shape
    l_max = int(case["l_max"])
    l_of_L = np.concatenate([[l] * (2 * l + 1) for l in range(l_max + 1)])
    A = coef[:, 0].reshape(n_at * n_l, n)
    B = coef[:, 1]
    norms = np.stack([case["udot_norm2"][int(case["atom_type"][a])][l_of_L] for a in range(n_at)])
    UB = (B * norms[:, :, None]).reshape(n_at * n_l, n)
    B = B.reshape(n_at * n_l, n)
    return A.conj().T @ A + B.conj().T @ UB


def hamiltonian(case: dict, coef: np.ndarray) -> np.ndarray:
    """H of Eq. 5: sum over atoms and (L', L) of the AA, AB, BA, BB terms with
    the type's T blocks.  The L-sum is taken first for each atom,
    Y_a = T_a [A_a; B_a] (associativity), then H = sum_a [A_a; B_a]^H Y_a as one
    product over the stacked index (a, A|B, L) (Eq. 6)."""
    n_at, _, n_l, n = coef.shape
    T = case["T"]
    Wst = coef.reshape(n_at, 2 * n_l, n)
    Y = np.stack([T[int(case["atom_type"][a])] @ Wst[a] for a in range(n_at)])
    return Wst.reshape(-1, n).conj().T @ Y.reshape(-1, n)


def hamiltonian_bruteforce(case: dict, coef: np.ndarray) -> np.ndarray:
    """Eq. 5 summed term by term with explicit loops (tiny inputs only)."""
    n_at, _, n_l, n = coef.shape
    H = np.zeros((n, n), dtype=np.complex128)
    for a in range(n_at):
        Tt = case["T"][int(case["atom_type"][a])]
        blocks = {("A", "A"): Tt[:n_l, :n_l], ("A", "B"): Tt[:n_l, n_l:],
                  ("B", "A"): Tt[n_l:, :n_l], ("B", "B"): Tt[n_l:, n_l:]}
        C = {"A": coef[a, 0], "B": coef[a, 1]}
        for gp in range(n):
            for g in range(n):
                acc = 0.0j
                for (x, y), Tb in blocks.items():
                    for lp in range(n_l):
                        for l in range(n_l):
                            acc += np.conj(C[x][lp, gp]) * Tb[lp, l] * C[y][l, g]
                H[gp, g] += acc
    return H


def hs(case: dict):
    """(H, S) full matrices for one k-point."""
    coef = coefficients(case)
    return hamiltonian(case, coef), overlap(case, coef)


def hs_entries(case: dict, rows: np.ndarray, cols: np.ndarray):
    """H[rows[i], cols[i]] and S[rows[i], cols[i]] for sampled index pairs,
    from the coefficients of only the G vectors involved."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    need, inv = np.unique(np.concatenate([rows, cols]), return_inverse=True)
    coef = coefficients(case, g=case["g"][need])
    ri, ci = inv[: len(rows)], inv[len(rows):]
    H = hamiltonian(case, coef)
    S = overlap(case, coef)
    return H[ri, ci], S[ri, ci]


def per_atom_blocks(case: dict, coef: np.ndarray):
    """Per-atom contributions H^a = W_a^H T_a W_a and S^a = W_a^H Lambda W_a."""
    n_at, _, n_l, n = coef.shape
    l_max = int(case["l_max"])
    l_of_L = np.concatenate([[l] * (2 * l + 1) for l in range(l_max + 1)])
    for a in range(n_at):
        t = int(case["atom_type"][a])
        Wa = coef[a].reshape(2 * n_l, n)
        lam = np.concatenate([np.ones(n_l), case["udot_norm2"][t][l_of_L]])
        yield a, Wa.conj().T @ (case["T"][t] @ Wa), Wa.conj().T @ (lam[:, None] * Wa)


def loss(case: dict, Wm: np.ndarray, Vm: np.ndarray, H=None, S=None) -> float:
    """L = Re tr(W H) + Re tr(V S)."""
    if H is None:
        H, S = hs(case)
    return float(np.real(np.sum(Wm * H.T)) + np.real(np.sum(Vm * S.T)))


def loss_gradients(case: dict, Wm: np.ndarray, Vm: np.ndarray):
    """Gradients of L = Re tr(W H) + Re tr(V S) with respect to T (per type,
    complex entries taken as free: grad = dL/dRe + i dL/dIm) and to the atom
    positions tau (cartesian).

    Route: every coefficient of atom a carries the phase e^{iK_G.tau_a}, so
    dH_{G'G}/dtau_a = i (K_G - K_G') H^a_{G'G} and likewise for S, with the
    per-atom blocks H^a, S^a; and L = Re sum_{ij} T_ij (W_a W W_a^H)_ji per atom."""
    coef = coefficients(case)
    n_at, _, n_l, n = coef.shape
    kvec = k_plus_g(case["lattice"], case["k_frac"], case["g"])
    grad_T = np.zeros_like(case["T"])
    grad_tau = np.zeros((n_at, 3))
    WmT = Wm.T
    VmT = Vm.T
    for a, Ha, Sa in per_atom_blocks(case, coef):
        t = int(case["atom_type"][a])
        Wa = coef[a].reshape(2 * n_l, n)
        grad_T[t] += Wa @ Wm.conj().T @ Wa.conj().T
        # sum over (G', G) of W_{G G'} i (K_G - K_G') H^a_{G' G}
        Ma = WmT * Ha + VmT * Sa  # [G', G]
        for c in range(3):
            dk = kvec[None, :, c] - kvec[:, None, c]
            grad_tau[a, c] = np.real(np.sum(1j * dk * Ma))
    return grad_T, grad_tau


def flops_forward(n_atoms: int, n_l: int, n_g: int) -> float:
    """Algorithmic FP64 flops of one H+S build: both upper triangles with the
    diagonal (2 N_at N_L complex multiply-adds per entry, 8 flops each) plus
    the per-atom T products (2N_L x 2N_L times 2N_L x N_G, complex)."""
    k_c = n_atoms * n_l
    return 16.0 * k_c * n_g * (n_g + 1) + 32.0 * n_atoms * n_l * n_l * n_g


def generalized_eigenvalues(H: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Eigenvalues, ascending, of the generalized problem H c = lambda S c that
    H and S are built for (Sec. 2.1), with S Hermitian positive definite: the
    library routine for the Hermitian-definite pencil (scipy.linalg.eigh)."""
    from scipy import linalg
    return linalg.eigh(H, S, eigvals_only=True)
