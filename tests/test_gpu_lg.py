"""GPU parity of the Laguerre-Gauss incident beams (sc_set_incident_lg, Sec. III-A) against the
oracle's independent generator: the aperture power per frequency, and the reflected field in FP64
(1e-12) and FP32-split (1e-5), for a linearly polarised higher-order mode (its current keeps one
direction per node: factored tables), a mixed superposition with circular polarisation (general
tables), and the radially polarised beam written as its LG_{0,+-1} combination.
"""
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


C01 = math.sqrt(2 / math.pi) / 15.0
AL = 1 / (2 * math.sqrt(2) * C01)
CASES = {
    "LG_1_2 x-polarised": ([(1, 2, 1.0, 0.0)], True),
    "LG_2_-1 polarised at 0.5 rad": ([(2, -1, math.cos(0.5), math.sin(0.5))], True),
    "superposition, circular part": ([(0, 0, 1.0, 0.0), (1, 1, 0.5, 0.5j), (0, -3, 0.2 - 0.1j, 0.0)], False),
    "radial beam from LG_0_+-1": ([(0, 1, AL, -1j * AL), (0, -1, AL, 1j * AL)], True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_lg_beam_matches_oracle(ctx, orc, name):
    from paper_1609_08146_amd import Problem
    modes, factors = CASES[name]
    f, a, nr, nphi, w0 = 20.0, 40.0, 90, 72, 15.0
    ks = np.array([K, 1.15 * K, 0.9 * K])
    spec = np.array([1.0, 0.6 - 0.3j, 0.8j])
    obs = workloads.random_points(96, 2.0, seed=12)
    m = orc.mirror(f, a, nr, nphi)
    Ei, Bi = orc.incident_lg_tables(m, ks, modes, w0, spec)
    Po = orc.incident_power(m, Ei, Bi)
    Eo, Bo = orc.reflected_field(m, ks, Ei, Bi, obs)
    p = Problem(ctx)
    p.set_mirror(f, a, nr, nphi)
    p.set_frequencies(ks)
    p.set_incident_lg(modes, w0, spec)
    p.set_observation(obs)
    P = p.incident_power()
    assert np.abs(P / Po - 1).max() < 1e-12, (P, Po)
    assert p.factored_for("fp32_split") is factors and p.factored_for("fp64") is factors
    errs = {}
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        errs[prec] = max(rel_l2(E, Eo), rel_l2(B, Bo))
        assert errs[prec] < tol, (prec, errs[prec])
    print(f"{name}: factored {factors}, power {np.abs(P / Po - 1).max():.1e}, "
          + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    if name.startswith("radial"):
        # the same field as the library's own radially polarised beam (different arithmetic path)
        q = Problem(ctx)
        q.set_mirror(f, a, nr, nphi)
        q.set_frequencies(ks)
        q.set_incident_beam("radial", w0, 0.0, spec, False)
        q.set_observation(obs)
        Er, Br = q.evaluate("fp64")
        E, B = p.evaluate("fp64")
        assert max(rel_l2(E, Er), rel_l2(B, Br)) < 1e-13
        q.close()
    p.close()


def test_lg_rejections(ctx):
    from paper_1609_08146_amd import Problem, ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL, SC_E_STATE
    p = Problem(ctx)
    with pytest.raises(ScError) as e:
        p.set_incident_lg([(0, 0, 1.0, 0.0)], 1.0)        # no mirror yet
    assert e.value.status == SC_E_STATE
    p.set_mirror(1.0, 1.0, 8, 8)
    p.set_frequencies([K])
    for modes, w0 in (([(-1, 0, 1.0, 0.0)], 1.0), ([(0, 65, 1.0, 0.0)], 1.0), ([(0, 0, float("nan"), 0.0)], 1.0),
                      ([(0, 0, 1.0, 0.0)], 0.0), ([(0, 0, 1.0, 0.0)], float("inf")), ([], 1.0)):
        with pytest.raises(ScError) as e:
            p.set_incident_lg(modes, w0)
        assert e.value.status == SC_E_INVAL
    p.close()
