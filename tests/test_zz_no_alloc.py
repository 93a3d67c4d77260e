"""sc_evaluate_noalloc, the evaluation entry point for callers that cannot allocate: its scratch
memory (work counters, job record, split-K partials) is a static device array, so the call allocates
nothing.  Through the C ABI it must give sc_evaluate's results bit for bit (same kernels, same node
chunks), on two calls in a row with the second problem smaller than the first (the array keeps the
first call's contents), in both split forms and on each table layout, and refuse cleanly when the problem's tables are not
built yet or its partials do not fit the array.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

# (enable factoring, tie the charge) per table layout
LAYOUTS = {"tied": (True, True), "factored": (True, False), "general": (False, True)}


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1609_08146_amd import Context
    c = Context(0)
    yield c
    c.close()


def _out(w, prec):
    import torch
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    shape = (w.n_k, w.n_obs, 3)
    return (torch.full(shape, complex("nan"), dtype=dt, device="cuda"),
            torch.full(shape, complex("nan"), dtype=dt, device="cuda"))


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("prec", ["fp32_split", "fp64"])
def test_noalloc_matches_evaluate_on_two_calls_in_a_row(ctx, prec, layout):
    from paper_1609_08146_amd import ScError, problem_from_workload
    from paper_1609_08146_amd._abi import SC_E_STATE
    big = workloads.broadband(n_k=8, n_nodes=96).subset(obs_idx=np.arange(0, 4160, 7))     # 595 points, 3 chunks
    small = workloads.mono().with_nodes(40, 32).subset(obs_idx=np.arange(0, 1024, 9))     # 114 points, 1 chunk
    probs, refs = [], []
    for w in (big, small):
        p = problem_from_workload(ctx, w)
        p.set_factoring(*LAYOUTS[layout])
        assert p.layout_for(prec) == layout, (w.name, prec)
        # the factored FP64 (and naive FP32) tables are built by the first evaluation in that precision:
        # before it, refused with nothing enqueued (the FP32-split tables of these beams exist already,
        # and so do the general FP64 ones, which the general layout reads as they are)
        for unbuilt in ("fp64", "fp32"):
            if unbuilt == prec or (unbuilt == "fp64" and layout == "general"):
                continue
            with pytest.raises(ScError) as e:
                p.evaluate_noalloc(_out(w, unbuilt), unbuilt)
            assert e.value.status == SC_E_STATE
        refs.append(p.evaluate(prec))
        probs.append(p)
    for w, p, (E0, B0) in zip((big, small), probs, refs):
        held = p.device_bytes()
        E, B = p.evaluate_noalloc(_out(w, prec), prec)
        ctx.synchronize()
        assert np.array_equal(E.cpu().numpy(), E0) and np.array_equal(B.cpu().numpy(), B0), (w.name, prec, layout)
        assert p.device_bytes() == held            # the problem's own buffers did not grow
        Er, Br = p.result()                         # the stored result is still sc_evaluate's
        assert np.array_equal(Er, E0) and np.array_equal(Br, B0)
    for p in probs:
        p.close()


def test_noalloc_refuses_partials_beyond_the_scratch(ctx):
    from paper_1609_08146_amd import ScError, problem_from_workload
    from paper_1609_08146_amd._abi import SC_E_INVAL, SC_NOALLOC_SCRATCH_BYTES
    w = workloads.broadband(n_k=16, n_nodes=400)    # partials 12 x 40 chunks x 16 x 4224 x 4 B = 130 MB
    p = problem_from_workload(ctx, w)
    E0, _ = p.evaluate("fp32_split")
    need = 12 * 40 * 16 * 4224 * 4
    assert need > SC_NOALLOC_SCRATCH_BYTES
    E, B = _out(w, "fp32_split")
    with pytest.raises(ScError) as e:
        p.evaluate_noalloc((E, B), "fp32_split")
    assert e.value.status == SC_E_INVAL and "scratch" in str(e.value)
    ctx.synchronize()
    assert bool(E.isnan().all())                    # nothing was written
    p.close()
