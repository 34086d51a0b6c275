"""The mixed-order batch entry point that allocates nothing
(sem_batch_rhs_static) against the plan-based one (sem_batch_plan +
sem_batch_execute, built-in tile shapes) through the C-ABI: the same values
bit for bit, and both within the forward gates of the oracle (FP64 1e-12,
FP32 2e-5 on the rounded inputs).  Two calls in a row, the second with fewer
blocks and elements, so the second runs on tables left by the first."""
import numpy as np
import pytest
import torch

from paper_1604_08501_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-5


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_08501_amd as m
    m.lib()
    return m


def _blocks(ws, dtype):
    cast = (lambda a: a) if dtype == torch.float64 else (lambda a: np.asarray(a, np.float32))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return [dict(q=dev(cast(w.q)), geo=dev(cast(w.geo)), D=dev(cast(w.D)),
                 rho_ref=dev(cast(w.rho_ref)), theta_ref=dev(w.theta_ref),
                 rhs=torch.full(w.q.shape, float("nan"), dtype=dtype, device="cuda"))
            for w in ws]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_rhs_static_matches_plan(sv, oracle_mod, dtype):
    tol = TOL64 if dtype == torch.float64 else TOL32
    for orders, per_order, k in (((1, 3, 5, 7, 9), 61, 400), ((2, 4), 9, 401)):
        ws = I.mixed_order_workloads(orders=orders, per_order=per_order, k=k)
        phys = ws[0].phys.as_tuple()
        blocks = _blocks(ws, dtype)
        plan = sv.BatchPlan(blocks, phys)
        plan.execute()
        torch.cuda.synchronize()
        ref = [b["rhs"].cpu().numpy().copy() for b in blocks]
        plan.close()
        for b in blocks:
            b["rhs"].fill_(float("nan"))
        sv.batch_rhs_static(blocks, phys)
        torch.cuda.synchronize()
        for w, b, r in zip(ws, blocks, ref):
            got = b["rhs"].cpu().numpy()
            assert np.array_equal(got, r), (orders, w.N)
            src = w if dtype == torch.float64 else I.upcast(I.to_fp32(w))
            o = oracle_mod.volume_rhs(src.D, src.geo, src.q, src.rho_ref, src.theta_ref, phys)
            e = I.rel_err_per_field(got, o)
            assert e.max() <= tol, (orders, w.N, e)


def test_batch_rhs_static_inside_a_captured_graph(sv):
    """The entry point without allocation records into a captured HIP graph
    (its fill kernel and the batch kernel); every replay, with a call of a
    different batch between replays rewriting the shared tables, equals the
    eager result bit for bit."""
    ws = I.mixed_order_workloads(orders=(2, 5, 8), per_order=23, k=402)
    other = I.mixed_order_workloads(orders=(3,), per_order=7, k=403)
    phys = ws[0].phys.as_tuple()
    blocks, others = _blocks(ws, torch.float64), _blocks(other, torch.float64)
    sv.batch_rhs_static(blocks, phys)
    torch.cuda.synchronize()
    eager = [b["rhs"].clone() for b in blocks]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            sv.batch_rhs_static(blocks, phys, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for replay in range(3):
        for b in blocks:
            b["rhs"].fill_(float("nan"))
        sv.batch_rhs_static(others, phys)              # rewrites the shared tables
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b, e in zip(blocks, eager):
            assert torch.equal(b["rhs"], e), replay


def test_batch_rhs_static_at_the_tile_limit(sv):
    """Exactly SEM_STATIC_MAX_TILES tiles (32768 tiles of the built-in FP64
    Nq = 4 shape, 8 elements each): the same bits as the plan-based entry
    point; one element more is rejected before any launch."""
    opts = sv.tile_options(torch.float64, 4)
    plan_probe = sv.BatchPlan(_blocks(I.mixed_order_workloads(orders=(3,), per_order=8, k=404),
                                      torch.float64), (1e5, 1.4, 287.0, 9.81))
    epb = plan_probe.describe()["orders"][0]["elems_per_block"]
    plan_probe.close()
    assert any(e == epb for e, _ in opts)
    Ne = 32768 * epb
    M = 64
    g = torch.Generator(device="cuda").manual_seed(405)
    rho = 1.0 + 0.01 * torch.rand(Ne, M, device="cuda", dtype=torch.float64, generator=g)
    q = torch.stack([rho] + [rho * 10 * (torch.rand(Ne, M, device="cuda", dtype=torch.float64,
                                                    generator=g) - 0.5) for _ in range(3)]
                    + [rho * 300.0], dim=1).contiguous()
    w1 = I.warped_workload(N=3, n_elements=1, k=406)
    geo = torch.from_numpy(w1.geo).cuda().expand(Ne, 10, M).contiguous()
    D = torch.from_numpy(w1.D).cuda()
    phys = w1.phys.as_tuple()
    blocks = [dict(q=q, geo=geo, D=D, rhs=torch.full_like(q, float("nan")))]
    plan = sv.BatchPlan(blocks, phys)
    assert plan.describe()["tiles"] == 32768
    plan.execute()
    torch.cuda.synchronize()
    ref = blocks[0]["rhs"].clone()
    plan.close()
    blocks[0]["rhs"].fill_(float("nan"))
    sv.batch_rhs_static(blocks, phys)
    torch.cuda.synchronize()
    assert torch.equal(blocks[0]["rhs"], ref)
    assert torch.isfinite(ref).all()
    over = [dict(q=torch.cat([q, q[:1]]), geo=torch.cat([geo, geo[:1]]), D=D,
                 rhs=torch.empty(Ne + 1, 5, M, dtype=torch.float64, device="cuda"))]
    with pytest.raises(sv.SemError, match="static tile table"):
        sv.batch_rhs_static(over, phys)
