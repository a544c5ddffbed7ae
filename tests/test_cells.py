"""The seeded input generator: reproducibility and the draw rules."""
import numpy as np
import pytest

from flapw_cells import CONFIGS, make_case, make_batch_case, basis_for_k


def test_reproducible():
    a = make_case(1, n_g=500)
    b = make_case(1, n_g=500)
    for key in ("tau", "radial", "udot_norm2", "T", "k_frac", "g"):
        np.testing.assert_array_equal(a[key], b[key])


def test_override_keeps_cell_draws():
    a = make_case(2, n_g=400)
    b = make_case(2, n_g=900)
    for key in ("tau", "radial", "udot_norm2", "T", "k_frac"):
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["g"], b["g"][:400])


@pytest.mark.parametrize("idx", [0, 1, 2, 4])
def test_rules(idx):
    cfg = CONFIGS[idx]
    c = make_case(idx, n_g=min(cfg.n_g, 1500))
    assert c["tau"].shape == (cfg.n_atoms, 3)
    assert np.all(np.diff(c["atom_type"]) >= 0)  # grouped by type
    lat = c["lattice"]
    frac = c["tau"] @ np.linalg.inv(lat)
    for i in range(cfg.n_atoms):
        d = frac[i] - frac[:i]
        d -= np.round(d)
        dist = np.linalg.norm(d @ lat, axis=1)
        ri = cfg.r_mt[c["atom_type"][i]]
        need = np.maximum(cfg.min_sep, ri + np.asarray(cfg.r_mt)[c["atom_type"][:i]])
        assert np.all(dist >= need - 1e-12)
    r = c["radial"]
    assert np.all((r >= 0.5) & (r <= 1.5))
    assert np.all(np.abs(r[..., 0] * r[..., 3] - r[..., 2] * r[..., 1]) >= 0.1)
    assert np.all((c["udot_norm2"] >= 0.01) & (c["udot_norm2"] <= 0.1))
    T = c["T"]
    assert T.shape == (cfg.n_types, 2 * cfg.n_l, 2 * cfg.n_l)
    np.testing.assert_array_equal(T, np.conj(np.transpose(T, (0, 2, 1))))
    d = np.real(np.diagonal(T, axis1=1, axis2=2))
    assert np.all(np.abs(d) <= 2)
    assert np.all(np.abs(c["k_frac"]) <= 0.5)


def test_basis_sorted_and_exact():
    c = make_case(1)
    assert len(c["g"]) == 3000
    bvec = 2 * np.pi * np.linalg.inv(c["lattice"]).T
    kn = np.linalg.norm((c["g"] + c["k_frac"]) @ bvec, axis=1)
    assert np.all(np.diff(kn) >= 0)
    assert kn[-1] < c["k_max"]
    # no lattice vector outside the list lies inside the cut-off sphere
    g2, _ = basis_for_k(c["lattice"], c["k_frac"], 3300)
    kn2 = np.linalg.norm((g2 + c["k_frac"]) @ bvec, axis=1)
    assert np.all(kn2[3000:] > c["k_max"])


def test_batch_case():
    b = make_batch_case(3, n_k=6)
    assert len(b["g"]) == 6 and b["k_frac"].shape == (6, 3)
    assert np.all((b["n_g"] >= 2800) & (b["n_g"] <= 3400))
    full = make_batch_case(3)
    assert len(full["g"]) == 64
    np.testing.assert_array_equal(full["n_g"][:6], b["n_g"])


def test_loss_matrices_hermitian():
    c = make_case(4, n_g=300)
    for key in ("W", "V"):
        M = c[key]
        assert M.shape == (300, 300)
        np.testing.assert_array_equal(M, M.conj().T)


def test_inversion_cells_are_paired():
    from flapw_cells import make_case
    for idx in (5, 6):
        case = make_case(idx, n_g=64)
        p, tau, t = case["partner"], case["tau"], case["atom_type"]
        assert np.array_equal(p[p], np.arange(len(p)))
        assert np.array_equal(t[p], t)
        assert np.abs(tau[p] + tau).max() == 0.0
        assert int((p == np.arange(len(p))).sum()) <= 1  # at most the origin atom
        # muffin tins keep the minimum separation, pairs included
        lat = case["lattice"]
        frac = tau @ np.linalg.inv(lat)
        for i in range(len(tau)):
            d = frac[i] - frac[i + 1:]
            d -= np.round(d)
            assert np.all(np.linalg.norm(d @ lat, axis=1) >= 3.0 - 1e-9)
