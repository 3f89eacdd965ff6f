"""Pins of the grid-spacing study's references: at grid nodes the
interpolated grid energy equals the direct pair sum with the grids'
exclusion (two independent codes: the C grid builder of Eq. 7 and the
numpy pair sum of Eqs. 4-6); trilinear interpolation is exact on affine
grids; far from every receptor atom exclusion changes nothing."""
import numpy as np
import pytest

import oracle
from oracle import pairs
from workload import synth


def _w():
    return synth.tiny(seed=4, n_rec=14, h=0.7, n_rec_atoms=40, n_lig_atoms=5, n_cfg=2, clash_mode="occ",
                      precision="f64")


def test_node_positions_grid_equals_direct_with_exclusion():
    w = _w()
    g, _ = oracle.receptor_grids(w)
    rng = np.random.default_rng(1)
    L = w.ligands[0]
    nodes = rng.integers(1, w.n_rec - 1, (6, L.n_atoms, 3))
    poses = w.origin[None, None, :] + w.h * nodes
    eg = pairs.grid_energies(g, w.h, w.origin, poses, L.q, L.sigma, L.eps)
    ed = pairs.pair_energies(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps, poses,
                             L.q, L.sigma, L.eps, exclusion=True)
    np.testing.assert_allclose(eg, ed, rtol=1e-11, atol=1e-9)


def test_trilinear_exact_on_affine_grid():
    n, h = 10, 0.5
    origin = np.array([1.0, -2.0, 0.5])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    a = np.array([0.3, -1.0, 2.0])
    b = np.array([[0.1, -0.2, 0.3], [1.0, 0.5, -0.25], [0.05, 0.0, 0.7]])   # per channel (bx, by, bz)
    g = np.stack([a[c] + b[c, 0] * x + b[c, 1] * y + b[c, 2] * z for c in range(3)])
    rng = np.random.default_rng(2)
    q, s, e = rng.normal(size=4), rng.uniform(3, 4, 4), rng.uniform(0.05, 0.2, 4)
    poses = origin + h * rng.uniform(0.5, n - 1.5, (3, 4, 3))
    got = pairs.grid_energies(g, h, origin, poses, q, s, e)
    gam = np.stack([q, np.sqrt(e) * s ** 6, -2 * np.sqrt(e) * s ** 3], axis=1)
    u = (poses - origin) / h
    want = np.stack([np.einsum("pi,i->p", a[c] + u @ b[c], gam[:, c]) for c in range(3)], axis=1)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-10)


def test_exclusion_is_inert_far_away():
    w = _w()
    L = w.ligands[0]
    poses = np.array([[[50.0 + i, 40.0, -30.0] for i in range(L.n_atoms)]])
    a = pairs.pair_energies(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps, poses,
                            L.q, L.sigma, L.eps, exclusion=True)
    b = pairs.pair_energies(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps, poses,
                            L.q, L.sigma, L.eps, exclusion=False)
    np.testing.assert_array_equal(a, b)
    # two point charges at 10 A: Coulomb's law
    one = pairs.pair_energies([[0, 0, 0]], [0.5], [3.0], [0.0], [[[10.0, 0, 0]]], [-0.4], [3.0], [0.0])
    assert one[0, 0] == pytest.approx(332.05 * 0.5 * -0.4 / 10.0, rel=1e-15)
    assert one[0, 1] == 0.0 and one[0, 2] == 0.0


def test_point_grid_values_equal_the_grid_builder():
    w = _w()
    g, o = oracle.receptor_grids(w)
    n = w.n_rec
    idx = np.random.default_rng(3).integers(0, n, (300, 3))   # (x, y, z)
    pts = w.origin[None, :] + w.h * idx
    r = w.receptor
    v = pairs.grid_values(r.xyz[0], r.q, r.sigma, r.eps, pts)
    want = np.stack([g[ch][idx[:, 2], idx[:, 1], idx[:, 0]] for ch in range(3)], axis=1)
    np.testing.assert_allclose(v, want, rtol=1e-12, atol=1e-12)
    occ = pairs.occupancy_values(r.xyz[0], r.sigma, w.occ_f, pts)
    np.testing.assert_array_equal(occ, o[idx[:, 2], idx[:, 1], idx[:, 0]])


def test_rasterised_occupancy_equals_the_grid_builder():
    w = _w()
    _, o = oracle.receptor_grids(w)
    r = w.receptor
    np.testing.assert_array_equal(pairs.occupancy_grid(r.xyz[0], r.sigma, w.occ_f, w.n_rec, w.h, w.origin), o)
