"""GPU parity of the built-in cylindrical vector beams (radially and
azimuthally polarised, Sec. IV-A) against the oracle, through the C ABI,
alone and through the serving loop."""
from dataclasses import replace

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


def _kind(orc, beam, consistent):
    return {(1, 0): orc.RADIAL, (1, 1): orc.RADIAL_CONSISTENT,
            (2, 0): orc.AZIMUTHAL, (2, 1): orc.AZIMUTHAL_CONSISTENT}[(beam, consistent)]


@pytest.mark.parametrize("beam,consistent", [(1, 0), (1, 1), (2, 0), (2, 1)])
def test_cylindrical_beam_field_matches_oracle(ctx, orc, beam, consistent):
    from paper_1609_08146_amd import problem_from_workload
    w = replace(workloads.broadband(n_k=6, n_nodes=90).subset(obs_idx=np.arange(0, 4160, 41)),
                beam=beam, consistent=consistent, w0=0.03)
    m = orc.mirror(w.f, w.a, w.n_r, w.n_phi)
    Ei, Bi = orc.incident_tables(m, w.k, _kind(orc, beam, consistent), w.w0, 0.0, w.spectrum)
    Eo, Bo = orc.reflected_field(m, w.k, Ei, Bi, w.obs)
    p = problem_from_workload(ctx, w)
    np.testing.assert_allclose(p.incident_power(), orc.incident_power(m, Ei, Bi), rtol=1e-13)
    for prec, tol in (("fp64", 1e-12), ("fp32_split", 1e-5)):
        E, B = p.evaluate(prec)
        err = max(rel_l2(E, Eo), rel_l2(B, Bo))
        print(f"beam {beam} consistent {consistent} {prec}: {err:.2e}")
        assert err < tol
    p.close()


def test_cylindrical_beam_rejections(ctx):
    from paper_1609_08146_amd import Problem, ScError
    from paper_1609_08146_amd._abi import SC_E_INVAL
    p = Problem(ctx)
    p.set_mirror(0.1, 0.075, 16, 16)
    p.set_frequencies([7.8e6])
    for beam, w0 in ((1, np.inf), (2, np.inf), (3, 0.05), (-1, 0.05), (1, 0.0)):
        with pytest.raises(ScError) as e:
            p.set_incident_beam(beam, w0)
        assert e.value.status == SC_E_INVAL
    p.set_incident_beam("radial", 0.05)
    p.close()


def test_served_radial_request_equals_single_solve(ctx):
    from paper_1609_08146_amd import Server, problem_from_workload
    w = replace(workloads.broadband(n_k=4, n_nodes=70).subset(obs_idx=np.arange(0, 4160, 97)), beam=1, w0=0.04)
    p = problem_from_workload(ctx, w)
    E0, B0 = p.evaluate("fp32_split")
    p.close()
    from paper_1609_08146_amd import Context
    c2 = Context(0, use_torch_stream=False)
    srv = Server(c2, hbm_budget=int(4e9), max_running=4, quantum_ms=5.0)
    try:
        t = srv.submit(w, "fp32_split")
        E, B, _, _, _ = srv.wait(t, timeout_ms=60000)
        assert np.array_equal(E, E0) and np.array_equal(B, B0)
    finally:
        srv.close()
        c2.close()
