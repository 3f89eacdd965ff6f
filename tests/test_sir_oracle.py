"""Pins of the oracle's pose resampling (sampling importance resampling):
on a grid of uniforms the draws of each level land on every configuration
and every translation with exactly the Boltzmann probabilities, whose
normalisations come from the pinned per-configuration BPMFs (Eq. 2)."""
import math

import numpy as np
import pytest

import oracle
from oracle import estimators as est
from workload import synth


def _setup():
    w = synth.tiny(seed=5, n_rec=12, h=1.0, n_rec_atoms=10, n_lig_atoms=2, n_cfg=4, clash_mode="occ", occ_f=0.3)
    go, oo = oracle.receptor_grids(w)
    parts, _ = oracle.scan(w, go, oo)
    cache = {}

    def energies(c):
        if c not in cache:
            r = oracle.config_eval(w, go, oo, 0, c)
            cache[c] = (r["psi"], r["clash"])
        return cache[c]
    return w, parts, energies


def test_configuration_level_frequencies():
    w, parts, energies = _setup()
    assert np.sum(parts[:, 3] > 0) >= 2
    M = 20000
    u1 = (np.arange(M) + 0.5) / M
    u = np.zeros(2 * M)
    u[0::2] = u1
    u[1::2] = 0.5
    cfg, _, _ = est.sample_poses(parts, energies, w.T, u)
    # Z_c = n_c exp(-B_c / kT), B_c the configuration's own Eq. 2 estimate
    Zc = np.array([parts[c, 2] * math.exp(-est.bpmf(parts[c:c + 1], w.T) / est.kT(w.T))
                   if parts[c, 3] > 0 else 0.0 for c in range(parts.shape[0])])
    freq = np.bincount(cfg, minlength=parts.shape[0]) / M
    assert np.max(np.abs(freq - Zc / Zc.sum())) <= 2.0 / M


def test_translation_level_frequencies():
    w, parts, energies = _setup()
    c = int(np.argmax(parts[:, 3]))
    # force the configuration: every other one gets nothing finite
    p1 = parts.copy()
    p1[np.arange(len(p1)) != c, 3] = 0
    psi, clash = energies(c)
    M = 50000
    u = np.zeros(2 * M)
    u[1::2] = (np.arange(M) + 0.5) / M
    cfg, t, ps = est.sample_poses(p1, energies, w.T, u)
    assert np.all(cfg == c)
    Vz, Vy, Vx = psi.shape
    lin = (t[:, 2] * Vy + t[:, 1]) * Vx + t[:, 0]
    np.testing.assert_allclose(ps, psi.ravel()[lin], rtol=0, atol=0)
    assert not np.any(clash.ravel()[lin])
    Zc = parts[c, 2] * math.exp(-est.bpmf(parts[c:c + 1], w.T) / est.kT(w.T))
    f = psi.ravel()
    ok = ~np.asarray(clash, bool).ravel()
    prob = np.where(ok, np.exp(-f / est.kT(w.T)), 0.0) / Zc
    assert prob.sum() == pytest.approx(1.0, rel=1e-12)
    freq = np.bincount(lin, minlength=f.size) / M
    assert np.max(np.abs(freq - prob)) <= 2.0 / M


def test_no_finite_translation_raises():
    w, parts, energies = _setup()
    p = parts.copy()
    p[:, 3] = 0
    with pytest.raises(ValueError):
        est.sample_poses(p, energies, w.T, np.full(4, 0.5))
