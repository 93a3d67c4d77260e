"""GPU: error of every output component against the oracle, for every form.

On the precision workload (f = 5 cm, aperture radius 15 cm, kR up to 1.6e6
rad, the full 800 x 800 nodes) at 64 points of the focal plane x 3
frequencies (band edges and carrier), each of E_x, E_y, E_z, B_x, B_y, B_z
gets two figures:

* the relative error of the paper's convergence study (Sec. IV-A, e_rel):
  max |F_c - F_c,ref| over points and frequencies divided by max |F_c,ref|,
  i.e. against the component's own peak, so weak cross-polarised components
  look worse;
* the same maximum error divided by the peak magnitude of the whole field
  (E or B), the figure the tolerances apply to.

Bounds: FP64 1e-12 and FP32-split (factored current and general tables)
1e-5 on the field-normalised maximum; the naive FP32 form (the whole phase
k|R| per pair in FP32) is at least 100 times worse than the split form.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

NAMES = ["E_x", "E_y", "E_z", "B_x", "B_y", "B_z"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


def component_errors(E, B, Eo, Bo):
    """[6] e_rel per component, [6] max error / peak |field| per component."""
    own, field = [], []
    for F, Fo in ((E, Eo), (B, Bo)):
        peak = float(np.max(np.linalg.norm(Fo, axis=-1)))
        for c in range(3):
            err = float(np.max(np.abs(F[..., c] - Fo[..., c])))
            own.append(err / float(np.max(np.abs(Fo[..., c]))))
            field.append(err / peak)
    return np.array(own), np.array(field)


def test_per_component_errors_on_the_precision_workload(ctx, orc):
    from paper_1609_08146_amd import problem_from_workload
    w = workloads.stress(n_k=64, n_nodes=800)
    sub = w.subset(obs_idx=np.arange(0, w.n_obs, 257), k_idx=[0, 31, 63])
    Eo, Bo = orc.solve(sub)
    p = problem_from_workload(ctx, sub)
    forms = {}
    for name, prec, fact, tie in (("fp64", "fp64", True, True), ("fp32_split tied", "fp32_split", True, True),
                                  ("fp32_split factored", "fp32_split", True, False),
                                  ("fp32_split general", "fp32_split", False, True), ("fp32 naive", "fp32", True, True)):
        p.set_factoring(fact, tie_charge=tie)
        E, B = p.evaluate(prec)
        forms[name] = component_errors(E, B, Eo, Bo)
    p.close()
    print(f"\n{sub.n_obs} points x {sub.n_k} frequencies x {sub.n_nodes} nodes; e_rel per component "
          f"(max error / component peak) and [max error / field peak]")
    print(f"{'form':22s}" + "".join(f"{n:>22s}" for n in NAMES))
    for name, (own, field) in forms.items():
        print(f"{name:22s}" + "".join(f"{o:>10.2e} [{f:8.2e}]" for o, f in zip(own, field)))
    assert forms["fp64"][1].max() < 1e-12
    assert forms["fp32_split tied"][1].max() < 1e-5
    assert forms["fp32_split factored"][1].max() < 1e-5
    assert forms["fp32_split general"][1].max() < 1e-5
    assert forms["fp32 naive"][1].max() > 100 * forms["fp32_split factored"][1].max()
