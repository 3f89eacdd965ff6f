"""The CPU FFT baseline (Eq. 9 through scipy.fft, FP64) against the direct
oracle: same partials of Eq. 2 per configuration, same energies at every
valid translation and the same clash set."""
import numpy as np

import oracle
from oracle import fft_cpu
from workload import synth


def _check(w, cfgs, psi_tol):
    g, occ = oracle.receptor_grids(w)
    spec = fft_cpu.receptor_spectra(w, g, occ)
    want, _ = oracle.scan(w, g, occ, 0, cfgs)
    L = w.ligands[0]
    gamma = oracle.ligand_weights(L)
    for i, c in enumerate(cfgs):
        p, psi, cl = fft_cpu.config_partial(w, spec, 0, int(c), return_fields=True)
        u, box = oracle.place_cfg(w, 0, int(c))
        direct = oracle.direct_energy(w, g, u, gamma, box)
        assert psi.shape == direct.shape
        assert np.linalg.norm(psi - direct) <= psi_tol * np.linalg.norm(direct)
        if occ is not None:
            np.testing.assert_array_equal(cl, oracle.clash(w, occ, u, oracle.occ_thresholds(L, w.occ_f, w.h), box))
        np.testing.assert_array_equal(p[[2, 3, 5]], want[i, [2, 3, 5]])  # counts and argmin
        fin = np.isfinite(want[i, [0, 1, 4]])
        np.testing.assert_allclose(p[[0, 1, 4]][fin], want[i, [0, 1, 4]][fin], rtol=1e-9, atol=1e-9)


def test_fft_cpu_matches_direct_cap_fp64():
    w = synth.config1()
    _check(w, np.arange(0, 100, 7), 1e-12)


def test_fft_cpu_matches_direct_occ_t4l_sized():
    w = synth.config2(n_rot=4, n_conf=1)
    _check(w, np.arange(2), 1e-11)
