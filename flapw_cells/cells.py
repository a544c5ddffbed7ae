"""Seeded synthetic cells: the five workload shapes and the draw rules.

Every array is drawn from numpy's PCG64 with seed 20171207 + config index, in
this order:

1. k: fractional coordinates uniform in [-1/2, 1/2)^3 (one row per k-point);
   for the multi-k workload, the per-k basis-size targets follow, uniform
   integers in the stated range;
2. atom positions, type-major, by random sequential addition: a uniform
   fractional position is redrawn until its minimum-image distance to every
   placed atom is at least max(min_sep, R_i + R_j);
3. radial boundary values per (type, l), in the order u, u', udot, udot',
   each uniform in [0.5, 1.5]; (udot, udot') is redrawn until the radial
   Wronskian |u udot' - udot u'| is at least 0.1;
4. ||udot_l||^2 per (type, l), uniform in [0.01, 0.1];
5. per type, the 2N_L x 2N_L Hermitian block T = [[T_AA, T_AB], [T_AB^H, T_BB]]:
   real diagonal uniform in [-2, 2], then the strictly upper triangle in
   row-major order as complex normals with E|z|^2 = 0.05^2 (real and
   imaginary parts each N(0, 0.05^2/2)); the lower triangle is the conjugate;
6. (loss workload only) W then V: Hermitian N_G x N_G, off-diagonal complex
   normal with E|z|^2 = 1/N_G^2, real diagonal N(0, 1/N_G^2).

Inversion-symmetric workloads (`inversion=True`) place each type's atoms as
pairs (tau, -tau) about the origin, the first atom of a type with an odd count
at the origin itself (at most one such type), so the positions are drawn one
per pair, and the distance rule covers both members.  Their T blocks come
from the same draws, made invariant under the two symmetries that make H and
S real: time reversal, T[(X,l,m),(X',l',m')] -> (-1)^(m+m') conj(T[(X,l,-m),(X',l',-m')])
(the block is replaced by the mean of itself and its image), and inversion
at the site, which removes the entries with l + l' odd.  `partner[a]` is the
atom paired with a (a itself at the origin).

The plane-wave basis of a k-point is the N_G reciprocal vectors G with the
smallest |k+G|, ties broken lexicographically on the integer triple; the
cut-off K_max is the midpoint between the N_G-th and (N_G+1)-th norms, so the
basis has exactly N_G members (the basis of Eq. 2 is all G with
|k+G| <= K_max).  That sorted order is the row and column order of H and S.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

SEED_BASE = 20171207


@dataclasses.dataclass(frozen=True)
class CellConfig:
    index: int
    name: str
    cell: tuple            # orthorhombic side lengths (bohr)
    atoms_per_type: tuple  # atoms of each type, types in order
    r_mt: tuple            # muffin-tin radius per type (bohr)
    l_max: int
    n_g: int = 0           # basis size of the single k-point
    n_k: int = 1
    ng_range: Optional[tuple] = None  # inclusive per-k basis-size range (multi-k)
    min_sep: float = 3.0
    with_loss: bool = False
    inversion: bool = False

    @property
    def n_types(self) -> int:
        return len(self.atoms_per_type)

    @property
    def n_atoms(self) -> int:
        return int(sum(self.atoms_per_type))

    @property
    def n_l(self) -> int:
        return (self.l_max + 1) ** 2


CONFIGS = {
    0: CellConfig(0, "cubic8_1x2_l4_ng256", (8.0, 8.0, 8.0), (2,), (1.2,), 4, n_g=256),
    1: CellConfig(1, "tet14x14x20_2x8_l8_ng3000", (14.0, 14.0, 20.0), (8, 8), (2.0, 2.3), 8, n_g=3000),
    2: CellConfig(2, "cubic30_4x32_l10_ng12000", (30.0, 30.0, 30.0), (32, 32, 32, 32),
                  (2.2, 2.2, 2.2, 2.2), 10, n_g=12000),
    3: CellConfig(3, "orth20x20x24_2x16_l8_64k", (20.0, 20.0, 24.0), (16, 16), (2.0, 2.3), 8,
                  n_k=64, ng_range=(2800, 3400)),
    4: CellConfig(4, "cubic24_2x32_l10_ng6000", (24.0, 24.0, 24.0), (32, 32), (2.2, 2.2), 10,
                  n_g=6000, with_loss=True),
    # inversion-symmetric cells (real-symmetric H and S)
    5: CellConfig(5, "cubic16_inv_2x8+7_l6_ng1500", (16.0, 16.0, 16.0), (8, 7), (1.8, 2.0), 6, n_g=1500,
                  inversion=True),
    6: CellConfig(6, "cubic30_inv_4x32_l10_ng12000", (30.0, 30.0, 30.0), (32, 32, 32, 32),
                  (2.2, 2.2, 2.2, 2.2), 10, n_g=12000, inversion=True),
    # edge cases: the largest l_max and type count the library takes; a type without atoms
    7: CellConfig(7, "cubic14_16x1_l12_ng400", (14.0, 14.0, 14.0), (1,) * 16, (1.2,) * 16, 12, n_g=400),
    8: CellConfig(8, "cubic12_inv_2+0+3_l3_ng300", (12.0, 12.0, 12.0), (2, 0, 3), (1.2, 1.3, 1.4), 3, n_g=300,
                  inversion=True),
}


def _lattice(cfg: CellConfig) -> np.ndarray:
    return np.diag(np.asarray(cfg.cell, dtype=np.float64))


def basis_for_k(lattice: np.ndarray, k_frac: np.ndarray, n_g: int):
    """The n_g reciprocal vectors with the smallest |k+G| (integer triples)
    and the midpoint cut-off K_max.  Returns (g int32[n_g,3], k_max)."""
    lattice = np.asarray(lattice, dtype=np.float64)
    k_frac = np.asarray(k_frac, dtype=np.float64)
    bvec = 2.0 * np.pi * np.linalg.inv(lattice).T  # rows b_j, a_i . b_j = 2 pi delta_ij
    omega = abs(np.linalg.det(lattice))
    k_est = (6.0 * np.pi ** 2 * n_g / omega) ** (1.0 / 3.0)
    radius = 1.25 * k_est + 1.0
    alen = np.linalg.norm(lattice, axis=1)
    while True:
        # (n + k)_i = K . a_i / (2 pi), so |n_i + k_i| <= |K| |a_i| / (2 pi)
        nmax = np.ceil(radius * alen / (2.0 * np.pi) + 1.0).astype(int)
        axes = [np.arange(-m, m + 1) for m in nmax]
        grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
        kvec = (grid + k_frac) @ bvec
        norm = np.sqrt(np.einsum("ij,ij->i", kvec, kvec))
        order = np.lexsort((grid[:, 2], grid[:, 1], grid[:, 0], norm))
        if len(order) > n_g and norm[order[n_g]] < radius:
            break
        radius *= 1.5
    k_lo, k_hi = norm[order[n_g - 1]], norm[order[n_g]]
    if not k_hi > k_lo:
        raise ValueError("tie at the basis cut-off: N_G=%d cannot be met exactly" % n_g)
    g = grid[order[:n_g]].astype(np.int32)
    return np.ascontiguousarray(g), 0.5 * (k_lo + k_hi)


def _min_image_ok(f, placed, lattice, need):
    if len(placed) == 0:
        return True
    d = f - np.asarray(placed)
    d -= np.round(d)
    return bool(np.all(np.linalg.norm(d @ lattice, axis=1) >= need))


def _place_pairs(rng, lattice, cfg: CellConfig):
    """Inversion-symmetric placement: per type, an atom at the origin if the
    count is odd, then pairs (f, -f) in consecutive slots."""
    radii = np.asarray(cfg.r_mt, dtype=np.float64)
    types, frac, partner, rads = [], [], [], []
    if sum(n % 2 for n in cfg.atoms_per_type) > 1:
        raise ValueError("%s: at most one type may have an atom at the origin" % cfg.name)
    for t, n in enumerate(cfg.atoms_per_type):
        if n % 2:
            need = np.maximum(cfg.min_sep, radii[t] + np.asarray(rads)) if rads else 0.0
            if not _min_image_ok(np.zeros(3), frac, lattice, need):
                raise RuntimeError("origin is occupied in %s" % cfg.name)
            partner.append(len(frac))
            types.append(t)
            frac.append(np.zeros(3))
            rads.append(radii[t])
        for _pair in range(n // 2):
            for _attempt in range(200000):
                f = rng.uniform(0.0, 1.0, 3)
                need = np.maximum(cfg.min_sep, radii[t] + np.asarray(rads)) if rads else 0.0
                d2 = (2.0 * f) - np.round(2.0 * f)  # separation of f and -f
                if (_min_image_ok(f, frac, lattice, need) and _min_image_ok(-f, frac, lattice, need)
                        and np.linalg.norm(d2 @ lattice) >= max(cfg.min_sep, 2 * radii[t])):
                    break
            else:
                raise RuntimeError("could not place a pair of type %d in %s" % (t, cfg.name))
            i = len(frac)
            partner.extend([i + 1, i])
            types.extend([t, t])
            frac.extend([f, -f])
            rads.extend([radii[t], radii[t]])
    return np.asarray(types, dtype=np.int32), np.asarray(frac) @ lattice, np.asarray(partner, dtype=np.int32)


def _symmetric_T(T, l_max):
    """The time-reversal mean and the site-inversion projection of a per-type
    Hermitian block on (A|B, l, m), L = l^2 + l + m."""
    n_l = (l_max + 1) ** 2
    lv = np.concatenate([[l] * (2 * l + 1) for l in range(l_max + 1)])
    mv = np.concatenate([np.arange(-l, l + 1) for l in range(l_max + 1)])
    flip = np.concatenate([lv * lv + lv - mv, n_l + lv * lv + lv - mv])  # index of (X, l, -m)
    sign = np.concatenate([(-1.0) ** mv, (-1.0) ** mv])
    ll = np.concatenate([lv, lv])
    out = []
    for A in T:
        image = sign[:, None] * sign[None, :] * np.conj(A[np.ix_(flip, flip)])
        B = 0.5 * (A + image)
        B[(ll[:, None] + ll[None, :]) % 2 == 1] = 0.0
        out.append(0.5 * (B + B.conj().T))
    return np.stack(out)


def _place_atoms(rng, lattice, cfg: CellConfig):
    types = np.repeat(np.arange(cfg.n_types, dtype=np.int32), cfg.atoms_per_type)
    radii = np.asarray(cfg.r_mt, dtype=np.float64)
    frac = np.zeros((len(types), 3))
    for i, t in enumerate(types):
        for _attempt in range(200000):
            f = rng.uniform(0.0, 1.0, 3)
            if i == 0:
                break
            d = f - frac[:i]
            d -= np.round(d)
            dist = np.linalg.norm(d @ lattice, axis=1)
            need = np.maximum(cfg.min_sep, radii[t] + radii[types[:i]])
            if np.all(dist >= need):
                break
        else:
            raise RuntimeError("could not place atom %d of %s" % (i, cfg.name))
        frac[i] = f
    return types, frac @ lattice


def _radial(rng, n_types, l_max):
    radial = np.zeros((n_types, l_max + 1, 4))
    for t in range(n_types):
        for l in range(l_max + 1):
            u, du, ud, dud = rng.uniform(0.5, 1.5, 4)
            while abs(u * dud - ud * du) < 0.1:
                ud, dud = rng.uniform(0.5, 1.5, 2)
            radial[t, l] = (u, du, ud, dud)
    return radial


def _hermitian_block(rng, m, diag_draw, sigma):
    diag = diag_draw(m)
    iu = np.triu_indices(m, 1)
    z = rng.normal(0.0, sigma / math.sqrt(2.0), (len(iu[0]), 2))
    a = np.zeros((m, m), dtype=np.complex128)
    a[iu] = z[:, 0] + 1j * z[:, 1]
    a = a + a.conj().T
    a[np.diag_indices(m)] = diag
    return a


def _draw(cfg: CellConfig, n_g_override: Optional[int]):
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + cfg.index))
    lattice = _lattice(cfg)
    k_frac = rng.uniform(-0.5, 0.5, (cfg.n_k, 3))
    targets = None
    if cfg.ng_range is not None:
        targets = rng.integers(cfg.ng_range[0], cfg.ng_range[1] + 1, cfg.n_k)
    partner = None
    if cfg.inversion:
        atom_type, tau, partner = _place_pairs(rng, lattice, cfg)
    else:
        atom_type, tau = _place_atoms(rng, lattice, cfg)
    radial = _radial(rng, cfg.n_types, cfg.l_max)
    udot_norm2 = rng.uniform(0.01, 0.1, (cfg.n_types, cfg.l_max + 1))
    m = 2 * cfg.n_l
    T = np.stack([_hermitian_block(rng, m, lambda n: rng.uniform(-2.0, 2.0, n), 0.05)
                  for _ in range(cfg.n_types)])
    if cfg.inversion:
        T = _symmetric_T(T, cfg.l_max)
    case = dict(
        name=cfg.name, config=cfg.index, lattice=lattice, omega=float(abs(np.linalg.det(lattice))),
        n_types=cfg.n_types, n_atoms=cfg.n_atoms, l_max=cfg.l_max, n_l=cfg.n_l,
        atom_type=atom_type.astype(np.int32), tau=np.ascontiguousarray(tau),
        r_mt=np.asarray(cfg.r_mt, dtype=np.float64), radial=radial, udot_norm2=udot_norm2,
        T=np.ascontiguousarray(T),
    )
    if partner is not None:
        case["partner"] = partner
    return rng, case, k_frac, targets


def make_case(index: int, n_g: Optional[int] = None) -> dict:
    """One k-point of workload `index`; `n_g` overrides the basis size (the
    cell, atoms, radial values and T are the same draws)."""
    cfg = CONFIGS[index]
    if cfg.n_k != 1:
        raise ValueError("config %d is a multi-k workload: use make_batch_case" % index)
    rng, case, k_frac, _ = _draw(cfg, n_g)
    n = int(n_g if n_g is not None else cfg.n_g)
    g, kmax = basis_for_k(case["lattice"], k_frac[0], n)
    case.update(k_frac=k_frac[0].copy(), g=g, n_g=n, k_max=kmax)
    if cfg.with_loss:
        sig = 1.0 / n
        case["W"] = _hermitian_block(rng, n, lambda k: rng.normal(0.0, sig, k), sig)
        case["V"] = _hermitian_block(rng, n, lambda k: rng.normal(0.0, sig, k), sig)
    return case


def make_batch_case(index: int = 3, n_k: Optional[int] = None) -> dict:
    """The multi-k workload: shared cell and T; per k its own basis, drawn
    with the per-k target size (K_max is therefore per k).  `n_k` keeps the
    first n_k k-points."""
    cfg = CONFIGS[index]
    rng, case, k_frac, targets = _draw(cfg, None)
    if targets is None:
        targets = np.full(cfg.n_k, cfg.n_g)
    use = cfg.n_k if n_k is None else int(n_k)
    gs, kmaxes = [], []
    for i in range(use):
        g, kmax = basis_for_k(case["lattice"], k_frac[i], int(targets[i]))
        gs.append(g)
        kmaxes.append(kmax)
    case.update(k_frac=np.ascontiguousarray(k_frac[:use]), g=gs,
                n_g=np.array([len(g) for g in gs], dtype=np.int32), k_max=np.array(kmaxes))
    return case


def sub_case(case: dict, k: int) -> dict:
    """The single-k view of k-point `k` of a multi-k case."""
    out = {key: val for key, val in case.items() if key not in ("k_frac", "g", "n_g", "k_max")}
    out.update(k_frac=case["k_frac"][k].copy(), g=case["g"][k], n_g=int(case["n_g"][k]),
               k_max=float(case["k_max"][k]))
    return out


def shell_sizes(lattice: np.ndarray, k_frac, upto: int):
    """The basis sizes up to `upto` at which the cut-off falls between two
    shells of |k+G| (the sizes basis_for_k accepts): at a high-symmetry k,
    such as k = 0, most sizes split a shell of equal norms."""
    lattice = np.asarray(lattice, dtype=np.float64)
    bvec = 2.0 * np.pi * np.linalg.inv(lattice).T
    omega = abs(np.linalg.det(lattice))
    radius = 1.5 * (6.0 * np.pi ** 2 * (upto + 1) / omega) ** (1.0 / 3.0) + 1.0
    nmax = np.ceil(radius * np.linalg.norm(lattice, axis=1) / (2.0 * np.pi) + 1.0).astype(int)
    grid = np.stack(np.meshgrid(*[np.arange(-m, m + 1) for m in nmax], indexing="ij"), axis=-1).reshape(-1, 3)
    kvec = (grid + np.asarray(k_frac, dtype=np.float64)) @ bvec
    norm = np.sort(np.sqrt(np.einsum("ij,ij->i", kvec, kvec)))
    assert norm[upto] < radius
    # norms of one shell can differ in the last bits (summation order): a gap must be real
    return [n for n in range(1, upto + 1) if norm[n] > norm[n - 1] * (1.0 + 1e-9)]


def at_k(case: dict, k_frac, n_g: Optional[int] = None) -> dict:
    """A copy of a single-k case moved to the k-point k_frac (reciprocal
    basis): the same cell, atoms, radial values and T, with the basis of that
    k chosen by the rule above (n_g must close a shell; see shell_sizes).
    The loss matrices of the loss workload are dropped."""
    n = int(case["n_g"] if n_g is None else n_g)
    kf = np.asarray(k_frac, dtype=np.float64).reshape(3).copy()
    g, kmax = basis_for_k(case["lattice"], kf, n)
    out = {key: val for key, val in case.items() if key not in ("W", "V")}
    out.update(k_frac=kf, g=g, n_g=n, k_max=kmax)
    return out


def perturb_positions(case: dict, delta: np.ndarray) -> dict:
    """A copy of `case` with tau replaced by tau + delta (cartesian)."""
    out = dict(case)
    out["tau"] = np.ascontiguousarray(case["tau"] + np.asarray(delta, dtype=np.float64))
    return out


def seeds(indices: Sequence[int]):
    return [SEED_BASE + i for i in indices]
