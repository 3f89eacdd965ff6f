"""Pins of the FP64 oracle against things other than itself: the pure-Python
restatement (brute force), closed forms, the correlation theorem through
numpy.fft, invariants and the constants printed in the paper."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from oracle import estimators as est
from workload import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _tiny(mode="occ", seed=3, n_rec=7, n_fft=None, n_lig=2, h=1.0, occ_f=0.5, **kw):
    w = synth.tiny(seed=seed, n_rec=n_rec, n_fft=n_fft, h=h, n_rec_atoms=5, n_lig_atoms=n_lig,
                   n_cfg=3, clash_mode=mode, occ_f=occ_f, **kw)
    return w


# ---------------------------------------------------------------- Eq. 7 grids
@pytest.mark.parametrize("mode", ["occ", "cap"])
def test_receptor_grids_match_brute(mode):
    w = _tiny(mode)
    g, occ = oracle.receptor_grids(w)
    r = w.receptor
    G, O = brute.receptor_grids(r.xyz[0].tolist(), r.q.tolist(), r.sigma.tolist(),
                                r.eps.tolist(), w.n_rec, w.h, w.origin.tolist(), mode,
                                w.ljr_cap, w.occ_f)
    G = np.array(G)
    np.testing.assert_allclose(g, G, rtol=1e-12, atol=1e-12)
    if mode == "occ":
        np.testing.assert_array_equal(occ, np.array(O, np.uint8))
        assert occ.sum() > 0


def test_ele_constant_and_exclusion_from_paper():
    """A single receptor atom: the ELE grid equals 332.05 q / r beyond the
    exclusion radius 2^-1/6 sigma and 0 inside (values printed in the paper)."""
    c = json.load(open(GOLD))
    k_ele = c["ele_kcal_per_e2_A"]["value"]
    f_ex = c["exclusion_radius_factor"]["value"]
    assert abs(f_ex - 2 ** (-1 / 6)) < 1e-15
    w = _tiny("occ", n_rec=9)
    w.receptor.xyz = np.array([[[0.3, -0.2, 0.1]]])
    w.receptor.q = np.array([0.7])
    w.receptor.sigma = np.array([3.5])
    w.receptor.eps = np.array([0.1])
    g, _ = oracle.receptor_grids(w)
    n = w.n_rec
    for (x, y, z) in [(0, 0, 0), (8, 8, 8), (4, 4, 4), (5, 4, 4), (2, 6, 1)]:
        p = w.origin + w.h * np.array([x, y, z])
        r = np.linalg.norm(p - w.receptor.xyz[0, 0])
        expect_ele = k_ele * 0.7 / r if r >= f_ex * 3.5 else 0.0
        se = math.sqrt(0.1)
        expect_ljr = se * 3.5 ** 6 / r ** 12 if r >= f_ex * 3.5 else 0.0
        expect_lja = se * 3.5 ** 3 / r ** 6 if r >= f_ex * 3.5 else 0.0
        idx = (z, y, x)
        assert g[0][idx] == pytest.approx(expect_ele, rel=1e-14, abs=1e-300)
        assert g[1][idx] == pytest.approx(expect_ljr, rel=1e-14, abs=1e-300)
        assert g[2][idx] == pytest.approx(expect_lja, rel=1e-14, abs=1e-300)
    assert np.any(g[0] == 0.0) and np.any(g[0] != 0.0)


def test_ligand_weights_eqs_4_to_6():
    c = json.load(open(GOLD))
    L = synth.tiny(seed=5).ligands[0]
    g = oracle.ligand_weights(L)
    se = np.sqrt(L.eps)
    np.testing.assert_allclose(g[:, 0], L.q, rtol=0, atol=0)
    np.testing.assert_allclose(g[:, 1], se * L.sigma ** c["lj_repulsive_sigma_power"]["value"], rtol=1e-15)
    np.testing.assert_allclose(g[:, 2], c["lj_attractive_ligand_factor"]["value"] * se *
                               L.sigma ** c["lj_attractive_sigma_power"]["value"], rtol=1e-15)
    # pair energy at the LJ minimum: gamma_i * receptor term = -eps_ij at r = sigma_ij
    # (r_min form: eps[(s/r)^12 - 2 (s/r)^6] has its minimum -eps at r = s)
    si, sj, ei, ej = 3.2, 3.7, 0.11, 0.07
    sij, eij = math.sqrt(si * sj), math.sqrt(ei * ej)
    r = sij
    e_r = math.sqrt(ei) * si ** 6 * math.sqrt(ej) * sj ** 6 / r ** 12
    e_a = -2 * math.sqrt(ei) * si ** 3 * math.sqrt(ej) * sj ** 3 / r ** 6
    assert e_r + e_a == pytest.approx(-eij, rel=1e-13)


# ---------------------------------------------------------------- placement
def test_placement_matches_quaternion_sandwich():
    w = synth.config2(n_rot=5, n_conf=2)
    L = w.ligands[0]
    for c in range(L.n_cfg):
        u, box = oracle.place_cfg(w, 0, c)
        ub, bb = brute.place(L.conformers[L.cfg_conf[c]].tolist(), L.cfg_quat[c].tolist(), w.h)
        assert np.max(np.abs(u - np.array(ub))) <= 2.0 ** -16
        assert list(box) == bb or np.max(np.abs(u - np.array(ub))) > 0


def test_rotation_convention_closed_forms():
    """Active rotation by the unit quaternion (cos t/2, sin t/2 n): a quarter
    turn about z takes x to y and y to -x; q and -q, and any positive
    multiple of q, rotate alike; a half turn about x negates y and z."""
    s = math.sqrt(0.5)
    qz = [s, 0.0, 0.0, s]
    np.testing.assert_allclose(brute.quat_rotate(qz, [1.0, 0.0, 0.0]), [0.0, 1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(brute.quat_rotate(qz, [0.0, 1.0, 0.0]), [-1.0, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(brute.quat_rotate([-3 * s, 0.0, 0.0, -3 * s], [0.3, -2.0, 1.5]),
                               brute.quat_rotate(qz, [0.3, -2.0, 1.5]), atol=1e-14)
    np.testing.assert_allclose(brute.quat_rotate([0.0, 1.0, 0.0, 0.0], [0.5, 2.0, -1.0]), [0.5, -2.0, 1.0],
                               atol=1e-15)
    # the C oracle places by the same convention: a two-atom rod along x,
    # turned a quarter about z, lies along y (3 A = 12 spacings at 0.25 A)
    rod = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0]])
    u, box = oracle.place(rod, np.array(qz), 0.25)
    np.testing.assert_allclose(np.sort(u[:, 1]), [2.0, 14.0], atol=2.0 ** -16)
    np.testing.assert_allclose(u[:, [0, 2]], 2.0, atol=2.0 ** -16)
    assert list(box) == [4, 16, 4]


def test_placement_invariants():
    c = json.load(open(GOLD))
    margin = c["placement_margin_spacings"]["value"]
    w = synth.config2(n_rot=20, n_conf=2)
    L = w.ligands[0]
    X = L.conformers[0]
    dref = np.linalg.norm(X[:, None] - X[None], axis=-1)
    for k in range(20):
        u, box = oracle.place(X, L.cfg_quat[k], w.h)
        # lowest coordinate exactly `margin` spacings from the 0 planes
        np.testing.assert_array_equal(u.min(axis=0), margin)
        # lattice
        np.testing.assert_array_equal(u * 65536, np.round(u * 65536))
        # box = ceil(max) + 2
        np.testing.assert_array_equal(box, np.ceil(u.max(axis=0)).astype(int) + c["ligand_box_margin_spacings"]["value"])
        # rigid: distances preserved up to the lattice rounding
        d = np.linalg.norm(u[:, None] - u[None], axis=-1) * w.h
        assert np.max(np.abs(d - dref)) < 2 * math.sqrt(3) * 2.0 ** -16 * w.h
        # q and -q are the same rotation
        u2, box2 = oracle.place(X, -L.cfg_quat[k], w.h)
        np.testing.assert_array_equal(u, u2)
        np.testing.assert_array_equal(box, box2)
    # identity quaternion: pure shift of the centred conformer
    u, _ = oracle.place(X, np.array([1.0, 0, 0, 0]), w.h)
    Y = X - X.mean(axis=0)
    expect = np.round(((Y - Y.min(axis=0)) / w.h + 2) * 65536) / 65536
    np.testing.assert_array_equal(u, expect)
    with pytest.raises(ValueError):
        oracle.place(X, np.zeros(4), w.h)


# ---------------------------------------------------------------- Eq. 8 directly
@pytest.mark.parametrize("mode,n_fft", [("occ", 7), ("cap", 7), ("occ", 10)])
def test_energy_and_clash_match_brute(mode, n_fft):
    w = _tiny(mode, n_rec=7, n_fft=n_fft, h=0.9, occ_f=0.35)
    g, occ = oracle.receptor_grids(w)
    L = w.ligands[0]
    G = g.tolist()
    gamma = oracle.ligand_weights(L)
    checked = 0
    for c in range(L.n_cfg):
        u, box = oracle.place_cfg(w, 0, c)
        if any(w.n_rec - b <= 0 for b in box):
            continue
        psi = oracle.direct_energy(w, g, u, gamma, box)
        ref = brute.energies(G, w.n_rec, w.n_fft, u.tolist(), gamma.tolist(), list(box))
        for (tx, ty, tz), v in ref.items():
            assert psi[tz, ty, tx] == pytest.approx(v, rel=1e-12, abs=1e-9)
            checked += 1
        if mode == "occ":
            thr = oracle.occ_thresholds(L, w.occ_f, w.h)
            cl = oracle.clash(w, occ, u, thr, box)
            rho = [w.occ_f * 2 ** (-1 / 6) * s / w.h for s in L.sigma]
            pts = brute.ligand_occ(u.tolist(), rho, w.n_fft)
            ov = brute.overlaps(occ.tolist(), w.n_rec, w.n_fft, pts, list(box))
            for (tx, ty, tz), v in ov.items():
                assert cl[tz, ty, tx] == (1 if v > 0 else 0)
    assert checked > 0


def test_single_point_charge_reproduces_grid():
    """gamma = (1,0,0) at integer u: Psi(t) = G_ELE(u + t) exactly."""
    rng = np.random.default_rng(0)
    w = synth.tiny(seed=1, n_rec=12, n_fft=16)
    g = rng.normal(size=(3, 12, 12, 12))
    u = np.array([[2.0, 3.0, 2.0]])
    box = np.array([4, 5, 4], np.int32)
    psi = oracle.direct_energy(w, g, u, np.array([[1.0, 0.0, 0.0]]), box)
    Vz, Vy, Vx = psi.shape
    expect = g[0][2:2 + Vz, 3:3 + Vy, 2:2 + Vx]
    np.testing.assert_array_equal(psi, expect)


def test_affine_grid_closed_form():
    """G_ch(n) = a_ch + b_ch . n (trilinear interpolation is exact):
    Psi(t) = sum_i sum_ch gamma_i,ch (a_ch + b_ch . (u_i + t))."""
    w = synth.config2(n_rot=3, n_conf=1)
    n = w.n_rec
    a = np.array([0.5, -1.0, 2.0])
    b = np.array([[0.1, -0.2, 0.3], [0.01, 0.02, -0.03], [1.0, 0.5, -0.25]])  # per ch: (bx,by,bz)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    g = np.stack([a[c] + b[c, 0] * x + b[c, 1] * y + b[c, 2] * z for c in range(3)])
    L = w.ligands[0]
    gamma = oracle.ligand_weights(L)
    u, box = oracle.place_cfg(w, 0, 1)
    psi = oracle.direct_energy(w, g, u, gamma, box)
    Vz, Vy, Vx = psi.shape
    for (tz, ty, tx) in [(0, 0, 0), (Vz - 1, Vy - 1, Vx - 1), (Vz // 2, 3, Vx // 3)]:
        t = np.array([tx, ty, tz])
        expect = sum(gamma[i, c] * (a[c] + b[c] @ (u[i] + t)) for i in range(L.n_atoms) for c in range(3))
        assert psi[tz, ty, tx] == pytest.approx(expect, rel=1e-12)


def test_linearity_and_translation_covariance():
    rng = np.random.default_rng(2)
    w = synth.tiny(seed=2, n_rec=14, n_fft=16)
    g = rng.normal(size=(3, 14, 14, 14))
    u = np.array([[2.0, 2.5, 3.25], [3.75, 2.0, 2.0]])
    box = np.ceil(u.max(axis=0)).astype(np.int32) + 2
    g1, g2 = rng.normal(size=(2, 3)), rng.normal(size=(2, 3))
    p1 = oracle.direct_energy(w, g, u, g1, box)
    p2 = oracle.direct_energy(w, g, u, g2, box)
    p12 = oracle.direct_energy(w, g, u, 2.0 * g1 - 3.0 * g2, box)
    np.testing.assert_allclose(p12, 2 * p1 - 3 * p2, rtol=1e-12, atol=1e-12)
    # shift all atoms by k=(1,2,1): Psi_shifted(t) = Psi(t + k)
    k = np.array([1, 2, 1])
    ps = oracle.direct_energy(w, g, u + k, g1, box + k)
    np.testing.assert_allclose(ps, p1[k[2]:, k[1]:, k[0]:], rtol=1e-13, atol=1e-13)


def test_correlation_theorem_fft_equals_direct():
    """Eq. 9 through numpy.fft (FP64) equals the direct sum of Eq. 8 at every
    box-valid translation, and the occupancy correlation gives the clash set."""
    w = synth.tiny(seed=4, n_rec=18, n_fft=24, h=0.7, n_rec_atoms=30, n_lig_atoms=3,
                   n_cfg=2, occ_f=0.5, r_ball=8.0)
    g, occ = oracle.receptor_grids(w)
    L = w.ligands[0]
    gamma = oracle.ligand_weights(L)
    thr = oracle.occ_thresholds(L, w.occ_f, w.h)
    N = w.n_fft
    pad = np.zeros((3, N, N, N))
    pad[:, :18, :18, :18] = g
    opad = np.zeros((N, N, N))
    opad[:18, :18, :18] = occ
    for c in range(L.n_cfg):
        u, box = oracle.place_cfg(w, 0, c)
        if any(w.n_rec - b <= 0 for b in box):
            continue
        direct = oracle.direct_energy(w, g, u, gamma, box)
        spec = np.zeros((N, N, N), complex)
        for ch in range(3):
            GL = oracle.spread_dense(N, u, gamma[:, ch])
            spec += np.fft.fftn(pad[ch]) * np.conj(np.fft.fftn(GL))
        C = np.real(np.fft.ifftn(spec))
        Vz, Vy, Vx = direct.shape
        fft_psi = C[:Vz, :Vy, :Vx]
        err = np.linalg.norm(fft_psi - direct) / np.linalg.norm(direct)
        assert err < 1e-12
        OL = oracle.occ_dense(N, u, thr)
        CO = np.real(np.fft.ifftn(np.fft.fftn(opad) * np.conj(np.fft.fftn(OL.astype(float)))))
        cl = oracle.clash(w, occ, u, thr, box)
        np.testing.assert_array_equal(CO[:Vz, :Vy, :Vx] > 0.5, cl.astype(bool))
        assert 0 < cl.sum() < cl.size


def test_zero_padding_invariance():
    w = synth.tiny(seed=6, n_rec=12, n_fft=12, h=0.8, n_rec_atoms=20, n_lig_atoms=2, n_cfg=2,
                   occ_f=0.3, r_ball=5.0)
    g, occ = oracle.receptor_grids(w)
    L = w.ligands[0]
    gamma = oracle.ligand_weights(L)
    u, box = oracle.place_cfg(w, 0, 0)
    a = oracle.direct_energy(w, g, u, gamma, box)
    w.n_fft = 20
    b = oracle.direct_energy(w, g, u, gamma, box)
    np.testing.assert_array_equal(a, b)


def test_occupancy_single_point_ball():
    """rho < 1/2 at an integer position: the ligand occupancy grid is the
    single point u, so clash(t) = O_R(u + t)."""
    rng = np.random.default_rng(9)
    w = synth.tiny(seed=1, n_rec=10, n_fft=12)
    occ = (rng.random((10, 10, 10)) < 0.3).astype(np.uint8)
    u = np.array([[2.0, 3.0, 2.0]])
    box = np.array([4, 5, 4], np.int32)
    thr = np.array([math.ceil(0.4 ** 2 * 2 ** 32)])
    cl = oracle.clash(w, occ, u, thr, box)
    Vz, Vy, Vx = cl.shape
    np.testing.assert_array_equal(cl, occ[2:2 + Vz, 3:3 + Vy, 2:2 + Vx])
    # a ball of radius exactly 1 holds the 7-point stencil minus nothing else
    pts = oracle.occ_dense(12, u, np.array([2.0 ** 32 + 1]))
    assert pts.sum() == 7


# ---------------------------------------------------------------- Eq. 2 partials
def test_partial_matches_numpy():
    rng = np.random.default_rng(1)
    psi = rng.normal(-5, 3, 1000)
    cl = (rng.random(1000) < 0.3).astype(np.uint8)
    beta = 1 / est.kT(300)
    p = oracle.partial(psi, cl, beta)
    fin = psi[cl == 0]
    assert p[2] == 1000 and p[3] == fin.size
    assert p[0] == pytest.approx(np.max(-beta * fin), rel=1e-15)
    assert p[1] == pytest.approx(np.sum(np.exp(-beta * fin - p[0])), rel=1e-13)
    assert p[4] == np.min(fin)
    assert int(p[5]) == int(np.flatnonzero((psi == np.min(fin)) & (cl == 0))[0])
    empty = oracle.partial(psi, np.ones(1000, np.uint8), beta)
    assert empty[3] == 0 and empty[1] == 0 and math.isinf(empty[4])


# ---------------------------------------------------------------- Eq. 2 / 12 / 13
T = 300.0


def _partials_from(psi_list, T=T):
    beta = 1 / est.kT(T)
    return np.array([oracle.partial(np.asarray(p, float), None, beta) for p in psi_list])


def test_bpmf_constant_energy():
    p = _partials_from([np.full(50, -3.2), np.full(70, -3.2)])
    assert est.bpmf(p, T) == pytest.approx(-3.2, abs=1e-12)


def test_bpmf_single_finite_sample():
    beta = 1 / est.kT(T)
    psi = np.array([-7.5, 1.0, 2.0, 3.0, 4.0])
    cl = np.array([0, 1, 1, 1, 1], np.uint8)
    p = np.array([oracle.partial(psi, cl, beta)])
    assert est.bpmf(p, T) == pytest.approx(-7.5 + est.kT(T) * math.log(5), abs=1e-12)
    # all clash -> +inf
    p = np.array([oracle.partial(psi, np.ones(5, np.uint8), beta)])
    assert math.isinf(est.bpmf(p, T))


def test_bpmf_bounds_and_naive():
    rng = np.random.default_rng(4)
    psis = [rng.normal(-4, 2, 200) for _ in range(6)]
    p = _partials_from(psis)
    B = est.bpmf(p, T)
    allpsi = np.concatenate(psis)
    assert allpsi.min() <= B <= allpsi.min() + est.kT(T) * math.log(allpsi.size)
    assert B == pytest.approx(est.bpmf_naive(allpsi, T), abs=1e-11)


def test_dg_closed_forms():
    kt = est.kT(T)
    vs = 1234.5
    # one snapshot
    assert est.dg_standard([-5.0], [1.0], vs, T) == pytest.approx(
        -5.0 - kt * math.log(vs * est.C_STANDARD), abs=1e-12)
    # equal B: independent of weights
    a = est.dg_standard([-2.0, -2.0, -2.0], [0.2, 0.3, 0.5], vs, T)
    b = est.dg_standard([-2.0, -2.0, -2.0], [0.6, 0.1, 0.3], vs, T)
    assert a == pytest.approx(b, abs=1e-12)
    # delta weights select one snapshot
    c = est.dg_standard([-2.0, -9.0, 3.0], [0.0, 1.0, 0.0], vs, T)
    assert c == pytest.approx(-9.0 - kt * math.log(vs * est.C_STANDARD), abs=1e-12)
    # standard state: 1 M is 1/1660.54 A^3
    assert 1.0 / est.C_STANDARD == pytest.approx(1660.539, rel=1e-6)


def test_vsite_counts():
    boxes = np.array([[40, 41, 42], [38, 38, 38]])
    v = est.v_site(boxes, 96, 0.25)
    assert v == pytest.approx(0.25 ** 3 * ((56 * 55 * 54) + 58 ** 3) / 2)


def test_is_estimators():
    rng = np.random.default_rng(5)
    lz = rng.normal(0, 2, 300)
    n_tot = 1e5
    Bfull = -est.kT(T) * (est.lse(lz) - math.log(n_tot))
    # uniform proposal, every configuration drawn once: exactly the full sum
    q = np.full(300, 1 / 300)
    assert est.bpmf_is(lz, n_tot, np.arange(300), q, T) == pytest.approx(Bfull, abs=1e-11)
    # unbiasedness of Z_hat under a skewed proposal (z-test over replicates)
    qq = est.proposal(lz + rng.normal(0, 0.5, 300), 0.1, 1.0)
    Z = np.exp(lz)
    vals = []
    for r in range(2000):
        idx = est.inverse_cdf_sample(qq, rng.random(20))
        vals.append(np.mean(Z[idx] / qq[idx]))
    vals = np.array(vals)
    z = (vals.mean() - Z.sum()) / (vals.std() / math.sqrt(len(vals)))
    assert abs(z) < 4


def test_proposal_mixture_closed_forms():
    """Defensive mixture q = (1 - alpha) softmax(yhat / tau) + alpha / P,
    checked against values worked out by hand."""
    # yhat = (0, ln 3): softmax = (1/4, 3/4); alpha = 0.2 -> 0.8 * (1/4, 3/4) + 0.1
    q = est.proposal(np.array([0.0, math.log(3.0)]), 0.2, 1.0)
    np.testing.assert_allclose(q, [0.3, 0.7], rtol=0, atol=1e-15)
    # tau divides the log weights: yhat = (0, 2 ln 3) at tau = 2 is the same mixture
    q2 = est.proposal(np.array([0.0, 2.0 * math.log(3.0)]), 0.2, 2.0)
    np.testing.assert_allclose(q2, [0.3, 0.7], rtol=0, atol=1e-15)
    # three configurations, yhat = (ln 1, ln 2, ln 5): softmax = (1/8, 2/8, 5/8)
    q3 = est.proposal(np.log([1.0, 2.0, 5.0]), 0.0, 1.0)
    np.testing.assert_allclose(q3, [0.125, 0.25, 0.625], rtol=0, atol=1e-15)
    # alpha = 1: uniform whatever the prediction
    y = np.random.default_rng(9).normal(0, 30, 50)
    np.testing.assert_allclose(est.proposal(y, 1.0, 0.7), np.full(50, 1 / 50), rtol=0, atol=1e-15)
    # a shift of every prediction leaves q unchanged; sum is one; floor alpha / P
    for alpha in (0.0, 0.1, 0.5):
        qa = est.proposal(y, alpha, 1.3)
        assert qa.sum() == pytest.approx(1.0, abs=1e-13)
        assert np.all(qa >= alpha / 50 - 1e-17)
        np.testing.assert_allclose(est.proposal(y + 123.0, alpha, 1.3), qa, rtol=1e-12)
    # huge predictions do not overflow (the softmax is max-shifted)
    qb = est.proposal(np.array([1000.0, 1000.0 - math.log(4.0)]), 0.0, 1.0)
    np.testing.assert_allclose(qb, [0.8, 0.2], rtol=0, atol=1e-14)


def test_inverse_cdf_sample():
    q = np.array([0.1, 0.2, 0.3, 0.4])
    u = np.array([0.0, 0.0999, 0.1000001, 0.2999, 0.3000001, 0.59, 0.61, 0.999999])
    np.testing.assert_array_equal(est.inverse_cdf_sample(q, u), [0, 0, 1, 1, 2, 2, 3, 3])


# ---------------------------------------------------------------- scan driver
def test_scan_driver_matches_per_config():
    w = synth.subset(synth.config1(), 6)
    g, occ = oracle.receptor_grids(w)
    parts, boxes = oracle.scan(w, g, occ, raw_everywhere=True)
    for c in range(6):
        r = oracle.config_eval(w, g, occ, 0, c)
        np.testing.assert_array_equal(parts[c], r["partial"])
        np.testing.assert_array_equal(boxes[c], r["box"])


def test_scan_occ_mode_skip_equals_raw():
    w = synth.tiny(seed=8, n_rec=16, n_fft=24, h=0.7, n_rec_atoms=40, n_lig_atoms=3, n_cfg=4,
                   r_ball=7.0)
    g, occ = oracle.receptor_grids(w)
    a, _ = oracle.scan(w, g, occ, raw_everywhere=True)
    b, _ = oracle.scan(w, g, occ, raw_everywhere=False)
    np.testing.assert_allclose(a, b, rtol=0, atol=0)
