"""The seeded synthetic inputs follow their stated recipe (CPU only): shapes
and sizes of the tiny, T4L-sized, batched and whole-surface workloads,
per-atom parameter ranges, ligand geometry (1.5 A bonds, 2.5 A non-bonded
separation, rigid pivot conformers), uniform unit quaternions, snapshot
jitter and weights, and determinism under the root seed."""
import numpy as np
import pytest

from workload import synth


@pytest.fixture(scope="module")
def c3():
    return synth.config3()


def _bonds_ok(xyz, parent, bond=1.5, min_sep=2.5):
    n = xyz.shape[0]
    d = np.linalg.norm(xyz[:, None] - xyz[None], axis=-1)
    bonded = np.zeros((n, n), bool)
    for i in range(1, n):
        p = parent[i]
        bonded[i, p] = bonded[p, i] = True
    iu = np.triu_indices(n, 1)
    return (np.allclose(d[bonded], bond, atol=1e-9)
            and bool(np.all(d[iu][~bonded[iu]] >= min_sep - 1e-9)))


def test_tree_and_pivot_conformers_keep_bonds_and_separation():
    rng = np.random.default_rng(5)
    for n in (2, 8, 25, 40):
        xyz, parent = synth.random_tree(rng, n)
        assert parent[0] == -1 and np.all(parent[1:] < np.arange(1, n))
        assert np.all(np.bincount(parent[1:], minlength=n) <= 3)   # at most three bonds each
        assert _bonds_ok(xyz, parent)
        confs = synth.pivot_conformers(rng, xyz, parent, 8)
        assert confs.shape == (8, n, 3)
        for k in range(8):
            assert _bonds_ok(confs[k], parent)
        if n >= 8:   # pivot moves change the shape
            assert np.max(np.abs(confs[-1] - confs[0])) > 0.1


def test_quaternions_are_unit_and_isotropic():
    q = synth.uniform_quaternions(np.random.default_rng(6), 200_000)
    np.testing.assert_allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-12)
    # uniform on the 3-sphere: E[q q^T] = I / 4
    np.testing.assert_allclose(q.T @ q / q.shape[0], np.eye(4) / 4, atol=5e-3)


def test_atom_parameter_ranges():
    q, s, e = synth.atom_params(np.random.default_rng(7), 100_000, synth.TINY_PARAMS)
    assert abs(q.std() - 0.4) < 0.01 and abs(q.mean()) < 0.01
    assert s.min() >= 3.0 and s.max() <= 4.0 and abs(s.mean() - 3.5) < 0.01
    assert e.min() >= 0.05 and e.max() <= 0.2
    q, s, e = synth.atom_params(np.random.default_rng(8), 100_000, synth.CAVITY_PARAMS)
    assert abs(q.std() - 0.1) < 0.005 and e.min() >= 0.025 and e.max() <= 0.1


def test_tiny_and_t4l_sized_workloads():
    w1 = synth.config1()
    assert (w1.n_rec, w1.n_fft, w1.h, w1.clash_mode, w1.precision) == (32, 32, 0.5, "cap", "f64")
    assert w1.receptor.xyz.shape == (1, 300, 3) and np.all(np.linalg.norm(w1.receptor.xyz[0], axis=1) <= 8.0)
    assert len(w1.ligands) == 1 and w1.ligands[0].n_atoms == 12 and w1.ligands[0].n_cfg == 100
    w2 = synth.config2()
    assert (w2.n_rec, w2.n_fft, w2.h, w2.clash_mode, w2.precision, w2.T) == (96, 128, 0.25, "occ", "f32", 300.0)
    r = np.linalg.norm(w2.receptor.xyz[0], axis=1)
    assert w2.receptor.xyz.shape == (1, 2600, 3) and r.min() >= 10.0 and r.max() <= 19.3
    L = w2.ligands[0]
    assert L.n_atoms == 25 and L.conformers.shape == (8, 25, 3) and L.n_cfg == 8000
    np.testing.assert_array_equal(np.bincount(L.cfg_conf), np.full(8, 1000))
    assert abs(L.q.sum()) < 1e-12                                   # a neutral ligand
    # the grid is centred on the cavity: its centre point sits at the origin
    np.testing.assert_allclose(w2.origin + 0.5 * (w2.n_rec - 1) * w2.h, 0.0, atol=1e-12)
    w6 = synth.config6(n_rot=10, n_conf=2)
    assert (w6.n_rec, w6.n_fft, w6.h) == (248, 256, 0.25) and w6.n_rec * w6.h == 62.0


def test_batched_workload(c3):
    rec = c3.receptor
    assert rec.xyz.shape == (10, 2600, 3)
    np.testing.assert_allclose(rec.weights, 0.1)
    # snapshots: the c2 receptor plus iid N(0, 0.3 A) per coordinate
    base = synth.config2(n_rot=1, n_conf=1).receptor.xyz[0]
    dev = rec.xyz - base[None]
    assert abs(dev.std() - 0.3) < 0.003 and abs(dev.mean()) < 0.003
    assert len(c3.ligands) == 141 and c3.n_cfg_total == 159504
    na = np.array([L.n_atoms for L in c3.ligands])
    nc = np.array([L.n_cfg for L in c3.ligands])
    assert na.min() >= 8 and na.max() <= 40
    assert np.all(nc % 8 == 0) and nc.min() >= 200 and nc.max() <= 2000
    assert all(L.conformers.shape[0] == 8 for L in c3.ligands)


def test_inputs_are_deterministic_under_the_root_seed():
    a, b = synth.config2(n_rot=20, n_conf=2), synth.config2(n_rot=20, n_conf=2)
    np.testing.assert_array_equal(a.receptor.xyz, b.receptor.xyz)
    np.testing.assert_array_equal(a.ligands[0].conformers, b.ligands[0].conformers)
    np.testing.assert_array_equal(a.ligands[0].cfg_quat, b.ligands[0].cfg_quat)
    c = synth.config2(seed=synth.ROOT_SEED + 1, n_rot=20, n_conf=2)
    assert not np.array_equal(a.receptor.xyz, c.receptor.xyz)
    np.testing.assert_array_equal(synth.uniforms(3, 10), synth.uniforms(3, 10))
