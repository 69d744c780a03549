"""GPU tests of the batched path: several vortex instances on meshes of uneven
size advanced together must equal each instance's plain path (same kernels,
same per-instance dt) bitwise, for every schedule and tile shape; HIP-graph
replays must equal eager steps (checked on every replay, with eager work and
synchronizations between replays); the dependency waits never time out."""
import numpy as np
import pytest
import torch

from paper_2102_12933_amd.inputs import batch_specs, make_mesh, vortex_state

pytestmark = pytest.mark.gpu


def _fdu():
    from paper_2102_12933_amd import fdu
    return fdu


def build_instances(specs, edge_variant=0, vertex_variant=0):
    fdu = _fdu()
    out = []
    for sp in specs:
        m = make_mesh(sp["N"], L=10.0, periodic=True, seed=sp["seed"])
        prep = fdu.Prep(m, deg=5, reorder=1)
        perm = prep.arrays()["perm"]
        s = fdu.Solver(prep, device=0)
        s.set_variants(edge_variant, vertex_variant)
        w0 = torch.from_numpy(vortex_state(m, beta=sp["beta"], mach=sp["mach"])[perm]).cuda()
        out.append((s, w0))
    return out


SPECS = [dict(N=N, seed=1000 + i, beta=b, mach=mc)
         for i, (N, b, mc) in enumerate([(33, 5.0, 0.5), (17, 3.0, 0.3), (48, 6.0, 0.8), (25, 2.0, 0.6), (40, 4.0, 0.45)])]


def plain_steps(inst, nsteps, cfl):
    outs = []
    for s, w0 in inst:
        w = w0.clone()
        scratch = torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda")
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        for _ in range(nsteps):
            s.rk_step(w, scratch, dt, cfl=cfl)
        outs.append(w.cpu())
    return outs


@pytest.mark.parametrize("edge_variant", [0, 1])
@pytest.mark.parametrize("schedule,ept,vp,vmode", [(0, 4, 8, 0), (0, 1, 1, 1), (0, 4, 8, 2), (1, 4, 8, 0),
                                                   (1, 16, 16, 2), (2, 4, 8, 0), (0, 16, 32, 0), (1, 4, 8, 3),
                                                   (1, 1, 1, 3), (2, 4, 8, 3), (0, 4, 8, 3), (0, 1, 1, 3)])
def test_batch_equals_plain(edge_variant, schedule, ept, vp, vmode):
    fdu = _fdu()
    # the plain path's vertex kernel with the same lanes and load order sums in the same order
    # the batch's lean edge phase is edge variant 1's code
    inst = build_instances(SPECS, edge_variant, vertex_variant=vmode)
    ref = plain_steps(inst, 3, 0.5)
    b = fdu.Batch([s for s, _ in inst])
    b.set_schedule(schedule, ept, vp, vmode)
    ws = [w0.clone() for _, w0 in inst]
    scr = [torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda") for s, _ in inst]
    b.set_states(ws, scr)
    for _ in range(3):
        b.step(0.5)
    err, dt = b.status()
    assert err == 0
    for i, (w, r) in enumerate(zip(ws, ref)):
        assert torch.equal(w.cpu(), r), (i, (w.cpu() - r).abs().max())


def test_batch_graph_replays_match_eager():
    fdu = _fdu()
    inst = build_instances(SPECS[:3])
    b = fdu.Batch([s for s, _ in inst])
    b.set_schedule(0, 4, 8, 0)
    ws = [w0.clone() for _, w0 in inst]
    scr = [torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda") for s, _ in inst]
    b.set_states(ws, scr)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b.capture(0.5, 2)
    torch.cuda.synchronize()
    state = [w0.clone() for _, w0 in inst]
    for rep in range(3):
        # eager reference from the same starting state
        ref = [x.clone() for x in state]
        for (s, _), x in zip(inst, ref):
            scratch = torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda")
            dt = torch.empty(1, dtype=torch.float64, device="cuda")
            for _ in range(2):
                s.rk_step(x, scratch, dt, cfl=0.5)
        for w, x in zip(ws, state):
            w.copy_(x)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            b.launch()
        side.synchronize()
        err, _ = b.status()
        assert err == 0
        for i, (w, r) in enumerate(zip(ws, ref)):
            assert torch.equal(w, r), (rep, i)
        state = [w.clone() for w in ws]
        _ = (state[0] * 2.0).sum().item()       # eager work between replays


def test_batch_table_matches_workload_description():
    specs = batch_specs()
    assert len(specs) == 64
    assert all(65 <= sp["N"] <= 513 and 2.0 <= sp["beta"] <= 6.0 and 0.3 <= sp["mach"] <= 0.8 for sp in specs)


def test_batch_set_schedule_rejects_bad_arguments():
    fdu = _fdu()
    inst = build_instances(SPECS[:2])
    b = fdu.Batch([s for s, _ in inst])
    for args in ((3, 4, 8, 0), (0, 0, 8, 0), (0, 4, 0, 0), (0, 4, 8, 4), (1, 65, 8, 0)):
        with pytest.raises(fdu.FduError, match="INVALID_ARG"):
            b.set_schedule(*args)
    b.set_schedule(0, 4, 8, 3)          # the fused schedule runs the LDS vertex blocks too
    with pytest.raises(fdu.FduError, match="INVALID_ARG"):
        fdu.Batch([])                   # an empty batch


@pytest.mark.slow
def test_full_batch_workload_sampled():
    """The batched workload at full size (64 instances, 7.0 M vertices, Hilbert
    order, the per-phase schedule with LDS vertex blocks and the fused
    persistent schedule): three steps at CFL 0.2 equal the plain path bit for
    bit on a sample of instances, and no dependency wait times out."""
    fdu = _fdu()
    specs = batch_specs(n=64)
    inst = []
    for sp in specs:
        m = make_mesh(sp["N"], L=10.0, periodic=True, seed=sp["seed"])
        prep = fdu.Prep(m, deg=5, reorder=2)
        perm = prep.arrays()["perm"]
        s = fdu.Solver(prep, device=0)
        w0 = torch.from_numpy(np.ascontiguousarray(vortex_state(m, beta=sp["beta"], mach=sp["mach"])[perm])).cuda()
        inst.append((s, w0))
    sample = [0, 17, 40, 63]
    for schedule, vmode, plain_vertex in ((1, 3, 3), (0, 2, 2), (0, 3, 3)):
        for s, _ in inst:
            s.set_variants(1, plain_vertex)
        ref = plain_steps([inst[i] for i in sample], 3, 0.2)
        b = fdu.Batch([s for s, _ in inst])
        b.set_schedule(schedule, 4 if schedule else 16, 8 if schedule else 16, vmode)
        ws = [w0.clone() for _, w0 in inst]
        scr = [torch.empty(2 * s.nv_total, 4, dtype=torch.float64, device="cuda") for s, _ in inst]
        b.set_states(ws, scr)
        for _ in range(3):
            b.step(0.2)
        err, _ = b.status()
        assert err == 0
        for k, i in enumerate(sample):
            assert torch.equal(ws[i].cpu(), ref[k]), (schedule, i)
        del b
