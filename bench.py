"""Benchmark: volume-RHS elements/s and GFLOP/s at N=7, FP64 and FP32.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the warped 32^3 box at N=7 (Nq=8, 512 nodes per element), 32768
curvilinear elements, 5 fields, D along r, s and t, gravity source and
reference-state pressure.  One step = one evaluation of the whole volume
term (one kernel launch over all elements) with inputs resident in HBM.
``value`` is the FP64 rate; the FP32 form of the same workload is reported
beside it, with its error against the FP64 oracle and the FP32/FP64 speedup.

Beside it the line carries the mixed-order batch (N = 3, 5, 7, 9,
5000 elements each; autotuned), one SSP-RK3 step replayed from a HIP graph
(stage updates fused into the batch launch, and as separate RHS + axpby
launches), and the adjoint (N=7, 8192 elements), each in FP64 and FP32, and
the paper-comparable configuration on the Table 2 shapes (FP32, 8 fields,
r+s and r+s+t, Nq = 4, 8, 12, 16 at 3,538,944 nodes) with the paper's own
timings on its hardware quoted beside it as context, and the per-element
metric form on an affine N=7 mesh of 32768 elements against the per-node
form of the same mesh, and the optimisation ladder of the paper's
benchmark kernel (levels 1-6) at Nq = 8 on the Table 2 shape.
Timing follows the paper's method (Sec. 4): after the warm-up launches every
leg keeps launching for at least 0.3 s, then times exactly ``--steps``
launches with HIP events on the launch stream; the mean per launch is the
reported rate (``ms_per_step``) and the median per launch is given beside it.

Prints one JSON line.  ``roofline`` prices the FP64 volume kernel against
the 8 TB/s HBM peak using the algorithmic bytes per node (176 B in FP64,
92 B in FP32); its duration is measured with HIP events on the launch
stream.  ``copy_reference`` is the rate of a plain 2 GiB device-to-device copy
on the same GPU, with the volume kernels' rates relative to it.
``cpu_baseline`` times the CPU oracle on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f64": 176, "f32": 92}


def flops_per_node(Nq: int) -> int:
    # 3 directions x 5 fields x Nq FMAs (2 FLOP each) + pointwise work
    # (1/rho 1, EOS/perturbation 6, fluxes 3 x 16, 1/J 5, source 3)
    return 30 * Nq + 63


# Sources that define the kernels whose measured traffic is recorded (the
# single-order volume and adjoint kernels, the extended kernels, the surface
# kernel and the whole-rate kernel).
VOLUME_KERNEL_SOURCES = ("sem_device.hpp", "sem_internal.hpp", "kernels.inc", "kernels_f64.hip",
                         "kernels_f32.hip", "ext.inc", "ext_f64.hip", "ext_f32.hip",
                         "surface.inc", "surface_f64.hip", "surface_f32.hip", "rhs.inc",
                         "rhs_f64.hip", "rhs_f32.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1604_08501_amd", "csrc")
    for f in VOLUME_KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key: str):
    """HBM bytes per launch from the committed PMC summary, if it was taken
    on the current kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    ent = d.get("kernels", {}).get(kernel_key)
    return ent.get("bytes_per_launch") if ent else None


def roof(gbs: float, key: str) -> dict:
    """Roofline record of one leg: its algorithmic GB/s against the HBM peak,
    and the HBM bytes per launch measured by PMC counters (or None)."""
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(key)}


# The paper's timing method (Sec. 4): after warm-up, keep launching for at
# least 0.3 s before the timed launches.  The shader clock ramps up over the
# first milliseconds of load after an idle spell (such as the host-side
# generation of a leg's inputs) and settles under sustained load, so every
# leg, the headline one included, times launches at the settled clock.
SETTLE_S = 0.3


def time_launches(fn, steps: int, warmup: int, stream, settle_s: float = SETTLE_S):
    """Warm up, keep launching for settle_s, then time exactly `steps`
    launches with one HIP event before each launch and one after the last,
    all on `stream`.  Returns (mean ms per launch, median ms per launch, wall
    seconds of the timed launches)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < settle_s:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i].record(stream)
        fn()
    ev[steps].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    mid = len(per) // 2
    median = per[mid] if len(per) % 2 else 0.5 * (per[mid - 1] + per[mid])
    return ev[0].elapsed_time(ev[steps]) / steps, median, wall


def copy_rate(gib: float, steps: int, warmup: int, stream, settle_s: float = SETTLE_S):
    """Rate of a plain device-to-device copy of `gib` GiB (bytes read + written
    over the launch time)."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    ms, _, _ = time_launches(lambda: dst.copy_(src), steps, warmup, stream, settle_s)
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 8, "ms": ms, "GBs": 2 * n * 8 / (ms * 1e-3) / 1e9}


def bench_batch_and_rk3(sv, I, steps: int, warmup: int, stream):
    """Mixed-order batch (N = 3, 5, 7, 9; 5000 warped elements each) as one
    launch, autotuned, and one SSP-RK3 step (dt = 1e-3) replayed
    from a HIP graph; FP64 and FP32.  Returns timings and algorithmic rates."""
    import torch
    ws = I.mixed_order_workloads()
    nodes = sum(w.Ne * w.Nq ** 3 for w in ws)
    out = {"workload": "N=3,5,7,9 x 5000 warped elements (8.96 M nodes)", "nodes": nodes}
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        cast = (lambda a: a) if dt == torch.float64 else (lambda a: np.asarray(a, np.float32))
        sizes = [w.q.size for w in ws]
        n = sum(sizes)
        q_n = torch.from_numpy(np.concatenate([cast(w.q).ravel() for w in ws])).cuda()
        q_1, q_2, L = (torch.empty_like(q_n) for _ in range(3))
        blocks, off = [], 0
        for w, sz in zip(ws, sizes):
            blocks.append(dict(q=q_n[off:off + sz].view(w.q.shape),
                               geo=torch.from_numpy(cast(w.geo)).cuda(),
                               D=torch.from_numpy(cast(w.D)).cuda(),
                               rho_ref=torch.from_numpy(cast(w.rho_ref)).cuda(),
                               theta_ref=torch.from_numpy(w.theta_ref).cuda(),
                               rhs=L[off:off + sz].view(w.q.shape)))
            off += sz
        plan = sv.BatchPlan(blocks, ws[0].phys.as_tuple(), autotune=True)
        ms_rhs, _, _ = time_launches(plan.execute, steps, warmup, stream)
        q0 = q_n.clone()
        bpn = BYTES_PER_NODE[tag]
        esz = 8 if tag == "f64" else 4
        rk = {}
        for mode, separate in (("fused", False), ("separate", True)):
            q_n.copy_(q0)
            g = sv.RK3Graph(blocks, q_n, q_1, q_2, L, 1e-3, ws[0].phys.as_tuple(), autotune=True,
                            separate_stages=separate)
            ms_rk, _, _ = time_launches(g.step, steps, warmup, stream)
            if separate:
                # 3 x (RHS + axpby); axpby reads 3 (2 in stage 1) and writes 1 value per dof
                rk_bytes = 3 * bpn * nodes + (4 + 4 + 3) * esz * n
            else:
                # 3 fused stages: RHS reads + stage-update writes, plus q_n in stages 2, 3
                rk_bytes = 3 * bpn * nodes + 2 * esz * n
            rk[mode] = {"step_ms": ms_rk, "GBs": rk_bytes / (ms_rk * 1e-3) / 1e9,
                        "bytes": rk_bytes}
            g.close()
        out[tag] = {"rhs_ms": ms_rhs, "rhs_el_s": sum(w.Ne for w in ws) / (ms_rhs * 1e-3),
                    "rhs_GBs": bpn * nodes / (ms_rhs * 1e-3) / 1e9, "rk3_step": rk,
                    "plan": plan.describe()}
        plan.close()
        del q_n, q_1, q_2, L, blocks
        torch.cuda.empty_cache()
    return out


def bench_adjoint(sv, I, steps: int, warmup: int, stream):
    """Vector-Jacobian product at N=7 on the first 8192 warped elements."""
    import torch
    w = I.adjoint_workload()
    nodes = w.Ne * w.Nq ** 3
    out = {"workload": "adjoint, N=7, 8192 warped elements", "nodes": nodes}
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        src = w if dt == torch.float64 else I.to_fp32(w)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        q, geo, D, lam = t(src.q), t(src.geo), t(src.D), t(src.lam)
        mu = torch.empty_like(q)
        ms, _, _ = time_launches(
            lambda: sv.volume_rhs_adjoint(q, geo, D, lam, w.phys.as_tuple(), out=mu),
            steps, warmup, stream)
        esz = 8 if tag == "f64" else 4
        gbs = 25 * esz * nodes / (ms * 1e-3) / 1e9
        out[tag] = {"ms": ms, "el_s": w.Ne / (ms * 1e-3), "GBs": gbs,
                    "roofline": roof(gbs, f"adjoint_{tag}_n7")}
    return out


# The paper's Table 2 (its level-8 kernel: FP32, 8 fields, r+s, rhsq
# accumulated) at a constant 3,538,944 nodes, for context; other hardware.
PAPER_TABLE2_MS = {
    4: {"R9 Fury X": 3.19944, "GTX Titan X": 1.78229, "Tesla K40c": 5.54140},
    8: {"R9 Fury X": 1.36146, "GTX Titan X": 2.06701, "Tesla K40c": 3.28739},
    12: {"R9 Fury X": 4.26229, "GTX Titan X": 2.20707, "Tesla K40c": 5.34723},
    16: {"R9 Fury X": 6.45935, "GTX Titan X": 2.11778, "Tesla K40c": 5.53732},
}


def bench_paper_table2(sv, I, steps: int, warmup: int, stream):
    """The paper-comparable configuration on the Table 2 shapes: 3,538,944 nodes
    at Nq = 4, 8, 12, 16 (Ne = 55296, 6912, 2048, 864) on a warped 2:2:1 box,
    FP32, 8 fields (3 passive tracers), the r and s terms only and with all
    three directions, the paper's constants (p0 = 1, gamma = 1.4, R = 1, no
    gravity, no reference state), rhs accumulated as in the listed kernels."""
    import torch
    phys = (1.0, 1.4, 1.0, 0.0)
    out = {"workload": "Table 2 shapes: 3,538,944 nodes, 8 fields, FP32, rhsq += v",
           "phys": phys}
    for Nq in (4, 8, 12, 16):
        w = I.to_fp32(I.table2_workload(Nq))
        nodes = w.Ne * Nq ** 3
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        q, geo, D = t(w.q), t(w.geo), t(w.D)
        rhs = torch.zeros_like(q)
        row = {"Ne": w.Ne, "paper_ms": PAPER_TABLE2_MS[Nq]}
        for name, dirs, geo_words in (("rs", 3, 7), ("rst", 7, 10)):
            ms, _, _ = time_launches(lambda: sv.volume_rhs_ext(q, geo, D, None, None, phys, dirs=dirs,
                                                               out=rhs, accumulate=True),
                                     steps, warmup, stream)
            # per node: q 8 + metric terms of the used directions and 1/J read,
            # rhs 8 read and 8 written, 4 bytes each
            byt = (8 + geo_words + 16) * 4 * nodes
            gbs = byt / (ms * 1e-3) / 1e9
            row[name] = {"ms": ms, "el_s": w.Ne / (ms * 1e-3), "GBs": gbs, "bytes": byt,
                         "roofline": roof(gbs, f"table2_{name}_nq{Nq}")}
        row["speedup_rs_vs_fury_x"] = PAPER_TABLE2_MS[Nq]["R9 Fury X"] / row["rs"]["ms"]
        out[f"Nq{Nq}"] = row
        del q, geo, D, rhs
        torch.cuda.empty_cache()
    return out


# The paper's Table 1 (its r+s, 8-field FP32 kernel at Nq = 8, Ne = 6910):
# wall time of its naive level 1 and its final level 8, in ms, for context.
PAPER_TABLE1_MS = {"R9 Fury X": (25.01630, 1.36121), "GTX Titan X": (7.17732, 2.06197),
                   "Tesla K40c": (14.29650, 3.28481)}


def bench_ladder(sv, I, steps: int, warmup: int, stream):
    """Optimisation ladder of the paper's benchmark kernel on the Table 2
    shape at Nq = 8 (6912 warped elements, 8 fields, FP32, r+s, rhs += v,
    p0 = 1, gamma = 1.4, R = 1): time per level and speedup over level 1."""
    import torch
    phys = (1.0, 1.4, 1.0, 0.0)
    w = I.to_fp32(I.table2_workload(8))
    nodes = w.Ne * w.Nq ** 3
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    q, geo, D = t(w.q), t(w.geo), t(w.D)
    rhs = torch.zeros_like(q)
    # the bytes the final kernel must move: q 8, metric terms 6 + 1/J, rhs 8
    # read and 8 written, 4 bytes each
    byt = (8 + 7 + 16) * 4 * nodes
    out = {"workload": f"Nq=8, {w.Ne} warped elements, 8 fields, FP32, r+s, rhsq += v",
           "paper_table1_ms_level1_level8": PAPER_TABLE1_MS, "levels": {}}
    base = None
    for level in range(1, sv.LADDER_LEVELS + 1):
        n_steps = steps if level >= 3 else max(3, steps // 10)
        ms, _, _ = time_launches(lambda: sv.volume_rhs_ladder(level, q, geo, D, phys, out=rhs),
                                 n_steps, min(warmup, 3) if level < 3 else warmup, stream,
                                 SETTLE_S if level >= 3 else 0.0)
        base = base or ms
        out["levels"][str(level)] = {"ms": ms, "speedup_vs_level1": base / ms,
                                     "GBs_final_kernel_bytes": byt / (ms * 1e-3) / 1e9}
    del q, geo, D, rhs
    torch.cuda.empty_cache()
    return out


def bench_affine(sv, I, steps: int, warmup: int, stream):
    """Per-element metric terms on an affine mesh: N=7, 32^3 = 32768 affine
    elements, FP64 and FP32, against the per-node form of the same mesh, and the optimisation ladder of the paper's
benchmark kernel (levels 1-6) at Nq = 8 on the Table 2 shape.
    The per-element form reads 10 words per element instead of 10 per node."""
    import torch
    w = I.affine_workload(N=7, n_side=32, k=1, with_adjoint=False)
    nodes = w.Ne * w.Nq ** 3
    out = {"workload": "N=7, 32768 affine elements (16.8 M nodes), 5 fields, r+s+t",
           "nodes": nodes}
    ge = I.element_geo(w.geo)
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        src = w if dt == torch.float64 else I.to_fp32(w)
        cast = (lambda a: a) if dt == torch.float64 else (lambda a: np.asarray(a, np.float32))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        q, geo, D, rr, tr = t(src.q), t(src.geo), t(src.D), t(src.rho_ref), t(src.theta_ref)
        g_el = t(cast(ge))
        o1, o2 = torch.empty_like(q), torch.empty_like(q)
        ph = w.phys.as_tuple()
        ms_node, _, _ = time_launches(lambda: sv.volume_rhs(q, geo, D, rr, tr, ph, out=o1),
                                      steps, warmup, stream)
        ms_elem, _, _ = time_launches(lambda: sv.volume_rhs_affine(q, g_el, D, rr, tr, ph, out=o2),
                                      steps, warmup, stream)
        torch.cuda.synchronize()
        diff = float(I.rel_err_per_field(o2.cpu().numpy(), o1.cpu().numpy()).max())
        esz = 8 if tag == "f64" else 4
        # per node: q 5 + rho_ref read, rhs 5 written (dtype) + theta_ref (FP64);
        # per element: 10 metric words
        byt = (11 * esz + 8) * nodes + 10 * esz * w.Ne
        gbs = byt / (ms_elem * 1e-3) / 1e9
        out[tag] = {"per_element_ms": ms_elem, "per_node_ms": ms_node,
                    "el_s": w.Ne / (ms_elem * 1e-3), "GBs": gbs,
                    "bytes": byt, "speedup_vs_per_node": ms_node / ms_elem,
                    "max_rel_diff_vs_per_node": diff, "roofline": roof(gbs, f"affine_{tag}_n7")}
        del q, geo, D, rr, tr, g_el, o1, o2
        torch.cuda.empty_cache()
    return out


def surface_bytes_per_element(Nq: int, esz: int) -> int:
    """Algorithmic bytes of the surface term per element (accumulating into
    rhs): at each of the Nb = Nq^3 - (Nq-2)^3 boundary nodes the state (5),
    1/J and rhs read and written (10) in the working precision and Theta_ref
    (8 B); at each of the 6 Nq^2 face-node pairs the three metric terms of the
    face direction; the six neighbour indices.  The neighbour's face values
    are its own boundary values, moved once."""
    nb = Nq ** 3 - max(Nq - 2, 0) ** 3
    return (16 * esz + 8) * nb + 3 * esz * 6 * Nq * Nq + 24


def rhs_bytes_per_element(Nq: int, tag: str) -> int:
    """Algorithmic bytes of the whole rate v + s per element: the volume
    term's inputs and outputs (the surface term's values are the same
    arrays, read once) and the six neighbour indices."""
    return BYTES_PER_NODE[tag] * Nq ** 3 + 24


def bench_surface(sv, I, w, steps: int, warmup: int, stream):
    """Surface term (strong-form DG face term, local Lax-Friedrichs flux) at
    N=7 on the periodic warped 32^3 box, accumulated into rhs; and the whole
    rate v + s, as the volume launch followed by the surface launch and as one
    launch."""
    import torch
    Ne, Nq = w.Ne, w.Nq
    out = {"workload": "surface term, N=7, 32768 warped elements, periodic, rhs += s",
           "bytes_per_element": {}}
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        src = w if dt == torch.float64 else I.to_fp32(w)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        q, geo, D, rr, tr, nbr = (t(src.q), t(src.geo), t(src.D), t(src.rho_ref),
                                  t(src.theta_ref), t(w.nbr))
        rhs = torch.zeros_like(q)
        ph = w.phys.as_tuple()
        ms, med, _ = time_launches(lambda: sv.surface_rhs(q, geo, nbr, tr, ph, out=rhs,
                                                          accumulate=True), steps, warmup, stream)

        def full():
            sv.volume_rhs(q, geo, D, rr, tr, ph, out=rhs)
            sv.surface_rhs(q, geo, nbr, tr, ph, out=rhs, accumulate=True)
        ms_full, _, _ = time_launches(full, steps, warmup, stream)
        # the whole rate in one launch: every input read once, rhs written once
        ms_one, med_one, _ = time_launches(
            lambda: sv.rhs(q, geo, D, nbr, rr, tr, ph, out=rhs), steps, warmup, stream)
        esz = 8 if tag == "f64" else 4
        bpe = surface_bytes_per_element(Nq, esz)
        gbs = bpe * Ne / (ms * 1e-3) / 1e9
        bpe_one = rhs_bytes_per_element(Nq, tag)
        gbs_one = bpe_one * Ne / (ms_one * 1e-3) / 1e9
        out["bytes_per_element"][tag] = bpe
        out[tag] = {"ms": ms, "median_ms": med, "el_s": Ne / (ms * 1e-3), "GBs": gbs,
                    "roofline": roof(gbs, f"surface_{tag}_n7"),
                    "volume_plus_surface_ms": ms_full,
                    "volume_plus_surface_el_s": Ne / (ms_full * 1e-3),
                    "one_launch": {"ms": ms_one, "median_ms": med_one, "el_s": Ne / (ms_one * 1e-3),
                                   "bytes_per_element": bpe_one, "GBs": gbs_one,
                                   "roofline": roof(gbs_one, f"rhs_{tag}_n7"),
                                   "speedup_vs_two_launches": ms_full / ms_one}}
        del q, geo, D, rr, tr, nbr, rhs
        torch.cuda.empty_cache()
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """What the host offers this process: the CPU count, the cores in its
    affinity mask and the OpenMP thread setting."""
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"nproc": os.cpu_count(), "affinity_cores": affinity,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle on the host cores (as many threads as OpenMP is given,
    the process's share of the host; then one) over the same N=7 workload: a
    reported baseline, not a target."""
    import oracle
    phys = w.phys.as_tuple()
    out = np.empty_like(w.q)
    oracle.volume_rhs(w.D, w.geo, w.q, w.rho_ref, w.theta_ref, phys, out=out)   # warm-up
    n, t0 = 0, time.perf_counter()
    while True:
        oracle.volume_rhs(w.D, w.geo, w.q, w.rho_ref, w.theta_ref, phys, out=out)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    cores = oracle.max_threads()
    # one core, on a 2048-element slice, for a short fixed budget
    oracle.set_threads(1)
    try:
        n1, t1 = 0, time.perf_counter()
        while True:
            oracle.volume_rhs(w.D, w.geo, w.q, w.rho_ref, w.theta_ref, phys, out=out,
                              elements=(0, 2048))
            n1 += 1
            el1 = time.perf_counter() - t1
            if el1 >= min(3.0, budget_s):
                break
    finally:
        oracle.set_threads(cores)
    return {"value": n * w.Ne / el, "unit": "elements/s", "cores": cores,
            "kind": "oracle", "cpu_model": _cpu_model(), "host": host_cores(),
            "value_1core": n1 * 2048 / el1,
            "sample": f"FP64 oracle over the full N=7 warped mesh ({w.Ne} elements), "
                      f"{n} passes in {el:.1f} s on {cores} threads; 1 thread: {n1} passes over "
                      f"the first 2048 elements in {el1:.1f} s"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mixed-order batch / RK3 graph, adjoint, Table 2 and affine measurements")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="only time a plain device-to-device copy of GIB GiB (the reference "
                         "for measured HBM bandwidth and for the PMC byte-counter scale)")
    ap.add_argument("--only", choices=("f64", "f32"), default=None,
                    help="time one precision only (profiling runs)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the volume term has no cross-GPU exchange, "
              "so a multi-GPU run is not part of this benchmark", file=sys.stderr)
        return 2

    import torch
    import oracle
    import paper_1604_08501_amd as sv
    from paper_1604_08501_amd import inputs as I

    sv.lib()   # raises if the HIP library is missing
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if a.copy_probe > 0:
        r = copy_rate(a.copy_probe, a.steps, a.warmup, stream)
        print(json.dumps({"copy_probe_bytes_read": r["bytes"] // 2, "copy_probe_bytes_written":
                          r["bytes"] // 2, "ms_per_copy": r["ms"], "copy_GBs": r["GBs"]}), flush=True)
        return 0

    t0 = time.perf_counter()
    w = I.warped_workload()                      # N=7, 32768 elements, seed k=2
    Ne, Nq = w.Ne, w.Nq
    nodes = Ne * Nq ** 3
    print(f"# generated workload in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    phys = w.phys.as_tuple()
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()

    results = {}
    ref64 = oracle.volume_rhs(w.D, w.geo, w.q, w.rho_ref, w.theta_ref, phys)
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        if a.only and tag != a.only:
            continue
        src = w if dt == torch.float64 else I.to_fp32(w)
        q, geo, D = dev(src.q), dev(src.geo), dev(src.D)
        rr, tr = dev(src.rho_ref), dev(src.theta_ref)
        out = torch.empty_like(q)
        fn = lambda: sv.volume_rhs(q, geo, D, rr, tr, phys, out=out)
        fn()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = ref64 if tag == "f64" else oracle.volume_rhs(
            *(np.asarray(x, np.float64) for x in (src.D, src.geo, src.q, src.rho_ref)),
            src.theta_ref, phys)
        err = float(I.rel_err_per_field(got, ref).max())
        ms, med, wall = time_launches(fn, a.steps, a.warmup, stream)
        bytes_launch = BYTES_PER_NODE[tag] * nodes
        results[tag] = dict(ms=ms, median_ms=med, wall=wall, err=err, bytes=bytes_launch,
                            el_s=Ne / (ms * 1e-3), gbs=bytes_launch / (ms * 1e-3) / 1e9,
                            gflops=flops_per_node(Nq) * nodes / (ms * 1e-3) / 1e9)
        print(f"# {tag}: {ms * 1e3:.1f} us/launch, {results[tag]['gbs']:.0f} GB/s, "
              f"err {err:.2e}", file=sys.stderr, flush=True)
        del q, geo, D, rr, tr, out
        torch.cuda.empty_cache()

    if a.only:
        r = results[a.only]
        print(json.dumps({"only": a.only, "ms_per_step": r["ms"], "GBs": r["gbs"],
                          "err": r["err"]}), flush=True)
        return 0
    r64, r32 = results["f64"], results["f32"]
    traffic = measured_traffic("volume_f64_n7")
    line = {
        # value: FP64 elements/s; GFLOP/s, the FP32 form and both errors beside it
        "metric": "volume-RHS elements/s and GFLOP/s at N=7, FP32 vs FP64 at stated error",
        "value": r64["el_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r64["ms"],
        "median_ms_per_step": r64["median_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded warped 32^3 mesh, random state about a hydrostatic reference)",
        "config": {"workload": "strong-form SEM volume RHS, N=7 (Nq=8), 32768 warped hex "
                               "elements, 5 fields, r+s+t, gravity, perturbation pressure",
                   "N": 7, "Ne": Ne, "nodes": nodes},
        "gflops": r64["gflops"],
        "err_fp64": r64["err"],
        "fp32": {"value": r32["el_s"], "unit": "elements/s", "ms_per_step": r32["ms"],
                 "median_ms_per_step": r32["median_ms"],
                 "gflops": r32["gflops"], "err_vs_fp64_oracle": r32["err"],
                 "roofline": {"bound": "hbm", "achieved": r32["gbs"], "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": r32["gbs"] / HBM_PEAK_GBS,
                              "traffic": measured_traffic("volume_f32_n7")}},
        "speedup_fp32_vs_fp64": r64["ms"] / r32["ms"],
        "roofline": {"bound": "hbm", "achieved": r64["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r64["gbs"] / HBM_PEAK_GBS, "traffic": traffic},
    }
    if not a.no_extra:
        # the same HBM moved by a plain device copy (read + write), for scale
        c = copy_rate(2.0, 20, 5, stream)
        line["copy_reference"] = {"workload": "device-to-device copy of 2 GiB", "GBs": c["GBs"],
                                  "f64_vs_copy": r64["gbs"] / c["GBs"],
                                  "f32_vs_copy": r32["gbs"] / c["GBs"]}
        line["surface"] = bench_surface(sv, I, w, a.steps, a.warmup, stream)
        line["batch_mixed_order"] = bench_batch_and_rk3(sv, I, a.steps, a.warmup, stream)
        line["adjoint"] = bench_adjoint(sv, I, a.steps, a.warmup, stream)
        line["paper_table2"] = bench_paper_table2(sv, I, a.steps, a.warmup, stream)
        line["affine_per_element"] = bench_affine(sv, I, a.steps, a.warmup, stream)
        line["opt_ladder"] = bench_ladder(sv, I, a.steps, a.warmup, stream)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
