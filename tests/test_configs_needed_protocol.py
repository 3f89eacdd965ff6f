"""The "configurations needed" protocol (CPU only): the replicate error
criterion, the plain and stratified K* searches and the per-snapshot scaling
of the exhaustive weights, pinned by cases whose answer is fixed by
construction (a flat pool, a zero-variance proposal, a known error).  The
stratified plan itself is the library's host routine (fftdg_is_plan), the
same one the measurement calls."""
import math

import numpy as np

from workload import synth

KT = 0.0019872041 * 300.0


def _err_rms(Zs, Zw):
    from paper_1708_07045_amd import proposal as prop
    return prop._err_rms(Zs, Zw, KT)


def test_replicate_error_is_the_free_energy_error():
    """kT ln(Z_hat / Z) per snapshot, RMS over replicates (bias included);
    an empty estimate counts as a failure (1e3 kcal/mol)."""
    rng = np.random.default_rng(1)
    Zs = rng.random((2, 50)) + 0.1
    Z = Zs.sum(axis=1)
    c = np.array([0.05, -0.2])                       # kcal/mol, one per snapshot
    Zw = np.tile(Z * np.exp(-c / KT), (7, 1))        # every replicate off by c
    np.testing.assert_allclose(_err_rms(Zs, Zw), np.abs(c), rtol=1e-12)
    # replicates +d and -d around the truth: RMS d, no bias to cancel it
    d = 0.08
    Zw = np.stack([Z * math.exp(-d / KT), Z * math.exp(d / KT)])
    np.testing.assert_allclose(_err_rms(Zs, Zw), [d, d], rtol=1e-12)
    Zw = np.stack([Z, np.zeros(2)])
    np.testing.assert_allclose(_err_rms(Zs, Zw), [1e3 / math.sqrt(2)] * 2, rtol=1e-12)


def test_plain_search_on_a_flat_pool_stops_at_the_first_size():
    """Equal weights: every uniform sample is exact, so K* is the distinct
    count of the first sample size (25 draws with replacement)."""
    from paper_1708_07045_amd import proposal as prop
    P = 500
    k = prop.kstar_plain(np.ones((3, P)), KT, np.random.default_rng(2), reps=40)
    assert prop.PLAIN_K[0] - 5 <= k <= prop.PLAIN_K[0]
    # one configuration holding all the weight in a small pool: the whole pool
    Zs = np.full((1, 40), 1e-30)
    Zs[0, 7] = 1.0
    assert prop.kstar_plain(Zs, KT, np.random.default_rng(3), reps=40) == 40.0


def _one_ligand_batch(P):
    import paper_1708_07045_amd as fd
    rng = np.random.default_rng(9)
    return fd.Batch([synth.make_ligand(rng, rng, 5, 1, P)])


def test_stratified_search_with_a_zero_variance_proposal():
    """With the proposal q proportional to Z (yhat = ln Z / 5 at a mixture
    temperature of 1 nat, alpha = 0, no exact stratum) every replicate is
    exact: K* is reached at the smallest budget, with at most that many
    distinct draws.  A temperature applied twice, a missing 1/q or a missing
    1/K would leave the heavy-tailed weights mis-estimated."""
    from paper_1708_07045_amd import proposal as prop
    P = 400
    b = _one_ligand_batch(P)
    rng = np.random.default_rng(4)
    lnZ = rng.normal(0.0, 3.0, P)
    Zs = np.exp(lnZ - lnZ.max())[None, :]
    y = (lnZ / 5.0).astype(np.float32)
    k, bf = prop.kstar_is(b, Zs, y, 0.0, 1.0, KT, 11, reps=30, exact_share=0.0)
    assert bf == prop.BUDGETS[0]
    assert 1 <= k <= math.ceil(prop.BUDGETS[0] * P)
    # the same proposal at 2 nats is no longer proportional to Z
    k2, bf2 = prop.kstar_is(b, Zs, y, 0.0, 2.0, KT, 11, reps=30, exact_share=0.0)
    assert bf2 is None or bf2 > prop.BUDGETS[0]


def test_stratified_search_with_the_whole_budget_exact():
    """A budget spent entirely on the exact top (nothing drawn) of a
    proposal that ranks the pool correctly: the estimate is the top's sum,
    so K* is the smallest budget whose ceil(bf P) largest weights hold
    enough of Z for the 0.1 kcal/mol criterion, found here by hand."""
    from paper_1708_07045_amd import proposal as prop
    P = 400
    b = _one_ligand_batch(P)
    rng = np.random.default_rng(5)
    lnZ = rng.normal(0.0, 4.0, P)
    Zs = np.exp(lnZ - lnZ.max())[None, :]
    y = (lnZ / 5.0).astype(np.float32)
    order = np.sort(Zs[0])[::-1]
    want = None
    for bf in prop.BUDGETS:
        nt = math.ceil(bf * P)
        if -KT * math.log(order[:nt].sum() / order.sum()) <= 0.1:
            want = (float(nt), bf)
            break
    assert want is not None and want[1] > prop.BUDGETS[0]
    assert prop.kstar_is(b, Zs, y, 0.1, 1.0, KT, 12, reps=5, exact_share=1.0) == want


def test_ligand_weights_scale_each_snapshot_to_its_maximum():
    """Z_{c,s} = s e^m scaled so the largest of each snapshot is 1; a
    configuration with nothing finite weighs 0."""
    from paper_1708_07045_amd import PARTIAL_DTYPE
    from paper_1708_07045_amd import proposal as prop
    P = np.zeros((2, 5), PARTIAL_DTYPE)
    lz = np.array([[3.0, 1.0, 0.0, 2.0, 0.0], [-7.0, -5.0, 0.0, -9.0, -6.0]])
    P["m"] = lz - math.log(2.0)
    P["s"] = 2.0
    P["n_finite"] = 1
    P["n_finite"][:, 2] = 0
    Z = prop.ligand_weights(P, [0, 2, 5], 1)          # ligand 1: configurations 2..4
    want = np.array([[0.0, 1.0, math.exp(-2.0)], [0.0, math.exp(-3.0), 1.0]])
    np.testing.assert_allclose(Z, want, rtol=1e-12, atol=0)
