"""Edge cases of the hot path against the oracle: degenerate mirrors, ragged
observation and frequency blocks, node chunks with a short tail, points at
the focus and on the axis, many frequencies, many points, and rejected sizes."""
import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
K = 2 * math.pi


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


def _problem(ctx, f, a, n_r, n_phi, ks, w0, obs, consistent=False):
    from paper_1609_08146_amd import Problem
    p = Problem(ctx)
    p.set_mirror(f, a, n_r, n_phi)
    p.set_frequencies(ks)
    p.set_incident_gaussian(w0, 0.0, None, consistent)
    p.set_observation(obs)
    return p


def _oracle(orc, f, a, n_r, n_phi, ks, w0, obs, consistent=False):
    m = orc.mirror(f, a, n_r, n_phi)
    kind = orc.PLANE if not np.isfinite(w0) else (orc.GAUSSIAN_CONSISTENT if consistent else orc.GAUSSIAN)
    Ei, Bi = orc.incident_tables(m, ks, kind, w0)
    return orc.reflected_field(m, ks, Ei, Bi, obs)


@pytest.mark.parametrize("n_r,n_phi", [(1, 1), (1, 2), (2, 3), (3, 1), (5, 4)])
def test_degenerate_mirrors(ctx, orc, n_r, n_phi):
    obs = np.array([[0.3, 0.2, 0.1], [0.0, 0.0, 0.0], [-1.0, 0.5, -0.7]])
    ks = [K, 1.3 * K, 0.8 * K]
    Eo, Bo = _oracle(orc, 20.0, 40.0, n_r, n_phi, ks, 20.0, obs)
    p = _problem(ctx, 20.0, 40.0, n_r, n_phi, ks, 20.0, obs)
    for opl, fpb in ((1, 1), (2, 1), (1, 4)):
        p.set_launch(obs_per_lane=opl, freq_per_lane=fpb, chunk=64)
        for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
            E, B = p.evaluate(prec)
            assert max(rel_l2(E, Eo), rel_l2(B, Bo)) < tol, (prec, opl, fpb)
    p.close()


@pytest.mark.parametrize("n_obs", [1, 63, 64, 65, 127, 129, 257])
def test_ragged_observation_blocks(ctx, orc, n_obs):
    rng = np.random.default_rng(n_obs)
    obs = rng.uniform(-2.0, 2.0, (n_obs, 3))
    ks = [K, 1.1 * K, 1.2 * K, 1.3 * K, 1.4 * K]        # 5: ragged blocks of 2 and 4 frequencies
    Eo, Bo = _oracle(orc, 20.0, 40.0, 9, 7, ks, 20.0, obs, consistent=True)
    p = _problem(ctx, 20.0, 40.0, 9, 7, ks, 20.0, obs, consistent=True)   # 70 nodes: chunks of 64 + 6
    for opl, fpb in ((1, 2), (2, 2), (1, 4)):
        p.set_launch(obs_per_lane=opl, freq_per_lane=fpb, chunk=64)
        E, B = p.evaluate("fp64")
        assert max(rel_l2(E, Eo), rel_l2(B, Bo)) < 1e-12, (opl, fpb)
        E, B = p.evaluate("fp32_split")
        assert max(rel_l2(E, Eo), rel_l2(B, Bo)) < 1e-5, (opl, fpb)
    p.close()


def test_focus_and_axis_points(ctx, orc):
    # the plane wave's focus closed form holds for the discrete sum: compare both sides there too
    f, a = 20.0, 25.0
    obs = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.4], [0.0, 0.0, -0.4]])
    Eo, Bo = _oracle(orc, f, a, 60, 32, [K], np.inf, obs)
    p = _problem(ctx, f, a, 60, 32, [K], np.inf, obs)
    E, B = p.evaluate("fp64")
    assert max(rel_l2(E, Eo), rel_l2(B, Bo)) < 1e-12
    U = a * a / (4 * f)
    ex = np.exp(2j * K * f) * (2j * K * f * U / (f + U) + U * (U - 2 * f) / (f + U) ** 2
                               - 2j * f * U / (K * (f + U) ** 3))
    assert abs(E[0, 0, 0] - ex) < 1e-9 * abs(ex)
    p.close()


def test_many_frequencies(ctx, orc):
    ks = K * np.linspace(0.5, 2.0, 1000)
    obs = np.array([[0.2, -0.1, 0.05], [0.0, 0.3, -0.2]])
    Eo, Bo = _oracle(orc, 20.0, 40.0, 12, 8, ks, 20.0, obs)
    p = _problem(ctx, 20.0, 40.0, 12, 8, ks, 20.0, obs)
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        assert max(rel_l2(E, Eo), rel_l2(B, Bo)) < tol, prec
    p.close()


def test_many_points_sampled(ctx, orc):
    n = 300_001
    rng = np.random.default_rng(5)
    obs = rng.uniform(-3.0, 3.0, (n, 3))
    p = _problem(ctx, 20.0, 40.0, 30, 24, [K], 20.0, obs)
    E, B = p.evaluate("fp32_split")
    idx = np.concatenate([[0, 1, n - 2, n - 1], rng.choice(n, 20, replace=False)])
    Eo, Bo = _oracle(orc, 20.0, 40.0, 30, 24, [K], 20.0, obs[idx])
    assert max(rel_l2(E[:, idx], Eo), rel_l2(B[:, idx], Bo)) < 1e-5
    p.close()


def test_rejected_sizes_and_empty_inputs(ctx):
    from paper_1609_08146_amd import Problem, ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL
    p = Problem(ctx)
    cases = [lambda: p.set_mirror(20.0, 40.0, 1 << 16, 1 << 15),     # (n_r + 1) n_phi >= 2^31 nodes
             lambda: p.set_mirror(20.0, 40.0, 0, 8),
             lambda: p.set_frequencies([]),
             lambda: p.set_observation(np.zeros((0, 3))),
             lambda: p.set_launch(chunk=100),
             lambda: p.set_frequencies(K * np.linspace(1.0, 2.0, 65536))]         # more than SC_MAX_FREQUENCIES
    for fn in cases:
        with pytest.raises(ScError) as e:
            fn()
        assert e.value.status == SC_E_INVAL
    p.close()
    p = _problem(ctx, 20.0, 40.0, 4, 4, [K], 20.0, np.zeros((1, 3)))
    p.evaluate("fp64")
    with pytest.raises(ScError) as e:
        p.to_time_at(1.0, np.zeros(524281))                                          # more than SC_MAX_TIMES
    assert e.value.status == SC_E_INVAL
    Et, _ = p.to_time_at(1.0, np.zeros(524280))
    assert Et.shape == (524280, 1, 3)
    p.close()
