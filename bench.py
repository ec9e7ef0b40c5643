#!/usr/bin/env python3
"""Throughput of the FP64 FMM gravity solve, forward + adjoint, at 128^3.

One step = one forward (rho -> phi, g) and one adjoint ((dphi, dg) -> drho)
of the whole 128^3 two-polytrope workload (uniform octree of depth 4, 4096
leaf sub-grids of 8^3 cells, theta = 0.4, order 3), inputs resident in HBM.

    python bench.py [--steps K] [--warmup W] [--cpu-slab Z]

Prints one JSON line.  `value` counts evaluated ordered cell pairs (leaf P2P
pairs plus M2L pairs of the coarser levels) per second over the K timed steps.
`roofline` reports the kernel with the largest share of GPU time (found in an
untimed pass that records every phase; the per-phase breakdown comes from that
pass), timed by HIP events around its launches inside the timed region, against
the FP64 vector peak of the MI355X.  `cpu_baseline` times the CPU
oracle (forward + adjoint) on a z-slab of the same workload.  `m2l_fp32` times
the FP32 M2L plan on the same workload; `batch` times 16 independent small
adaptive octrees plan by plan, as one batch over 4 streams and as HIP graph replays;
`amr` times the adaptive-octree workload (leaves on levels 3..6 of a 512^3
box) and, in the CPU-baseline leg, checks sampled cells against the oracle;
`am_correction` times the angular-momentum correction at 128^3 and reports
the total torque with and without it.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12       # MI355X FP64 vector: 256 CU x 128 FLOP/clk x 2.4 GHz
METRIC = "cell-interactions/s & FP64 FLOP/s (fwd+adjoint) at 128³ vs FP64 peak; oracle err"
# FP64 FLOP the kernels issue per algorithmic FLOP: the M2L evaluates the
# contraction in its traceless-reduced form, 70 FMA per pair instead of 84
ISSUED_PER_ALGORITHMIC = {"m2l": 140.0 / 168.0}
# kernel of each phase at depth >= 2 (depths 0 and 1 run k_upward_leaf for the upward phases)
KERNEL_OF_PHASE = {"m2l": "k_m2l", "leaf": "k_leaf<false>", "leaf_adj": "k_leaf<true>",
                   "upward_leaf": "k_m2m_span<1>", "upward_leaf_adj": "k_m2m_span<2>",
                   "m2m": "k_m2m_span<0>", "l2l": "k_l2l_span"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ot_fmm_kernels.hip", "ot_fmm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2412_15518_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(phase: str):
    """HBM traffic per launch from a committed rocprofv3 PMC summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{phase}_traffic_128.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != kernel_source_hash():
        return None
    return float(b.group(1))


def phase_flops(phase: str, info: dict) -> float:
    """Algorithmic FLOP of one launch group of a phase.  The upward phases
    hold the P2M and the M2M of the levels up to three above the leaves
    (cells of levels max(1, L-4)..L-1 are shifted to their parents); the
    m2m phase holds the rest; the l2l phase the shifts into levels 1..L-2
    (the leaf phases form level L-1)."""
    N = info["n_leaf_cells"]
    L = info["depth"]
    cells = lambda lo, hi: sum((8 << l) ** 3 for l in range(lo, hi))   # noqa: E731
    m2m_low = 168.0 * cells(max(1, L - 4), L)
    return {"m2l": 168.0 * info["m2l_pairs"],
            "leaf": 8.0 * info["p2p_pairs"] + 100.0 * N + 168.0 * cells(L - 1, L),
            "leaf_adj": 8.0 * info["p2p_pairs"] + 40.0 * N + 168.0 * cells(L - 1, L),
            "upward_leaf": 40.0 * N + m2m_low,
            "upward_leaf_adj": 100.0 * N + m2m_low,
            "m2m": 168.0 * cells(1, max(1, L - 4)),
            "l2l": 168.0 * cells(1, L - 1)}[phase]


def bench_batch(args) -> dict:
    """16 independent adaptive octrees (leaf sub-grid targets log-uniform in
    [64, 1024], seed 3, grown by density-ranked refinement and balanced 2:1):
    forward + adjoint of all of them per step, plan by plan on one stream, as
    one batch over 4 streams, and as the replay of that batch captured in two
    HIP graphs."""
    import numpy as np
    import torch

    from paper_2412_15518_amd import fmm, workloads as W
    trees = W.batch_of_octrees()
    plans, rhos, ws, us, phis, gs, drhos = [], [], [], [], [], [], []
    pairs = 0
    for t in trees:
        p = fmm.Plan(t["layout"])
        inf = p.info()
        pairs += 2 * (inf["p2p_pairs"] + inf["m2l_pairs"])
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
        plans.append(p)
        rhos.append(dev(t["rho"]))
        ws.append(dev(t["w"]))
        us.append(dev(t["u"]).reshape(-1))
        phis.append(torch.empty_like(rhos[-1]))
        gs.append(torch.empty(3 * rhos[-1].numel(), dtype=torch.float64, device="cuda"))
        drhos.append(torch.empty_like(rhos[-1]))
    ns = 4
    b = fmm.Batch(plans, n_streams=ns)
    gf = b.capture_forward(rhos, phis, gs)
    ga = b.capture_adjoint(ws, us, drhos)

    def single():
        for i, p in enumerate(plans):
            p.forward_into(rhos[i], phis[i], gs[i])
            p.adjoint_into(ws[i], us[i], drhos[i])

    def batched():
        b.forward_into(rhos, phis, gs)
        b.adjoint_into(ws, us, drhos)

    def graphs():
        gf.launch()
        ga.launch()

    k = max(5, min(args.steps, 50))
    res = {}
    outs = {}
    for name, fn in (("single", single), ("batch", batched), ("graph", graphs)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        res[name] = 1e3 * (time.perf_counter() - t0) / k
        outs[name] = [x.clone() for x in phis + gs + drhos]
    same = all(torch.equal(a, c) for n in ("batch", "graph") for a, c in zip(outs[n], outs["single"]))
    gf.close()
    ga.close()
    b.close()
    log(f"batch of {len(trees)} trees: single {res['single']:.3f} ms, batch {res['batch']:.3f} ms, "
        f"graph {res['graph']:.3f} ms per step")
    return {"workload": f"{len(trees)} adaptive octrees, leaf sub-grid targets log-uniform in [64, 1024] (seed 3), "
                        f"grown by density-ranked refinement of a sphere or polytrope, 2:1 balanced, depths "
                        f"{sorted(set(t['layout'].depth for t in trees))}, {sum(t['n_leaf'] for t in trees)} leaf "
                        f"sub-grids; one step = forward + adjoint of every tree",
            "steps": k, "streams": ns, "cell_interactions_per_step": pairs,
            "ms_per_step": res, "cell_interactions_per_s_graph": pairs / (res["graph"] * 1e-3),
            "speedup_graph_vs_single": res["single"] / res["graph"],
            "speedup_batch_vs_single": res["single"] / res["batch"],
            "outputs_identical": same}


def bench_amr(args):
    """The adaptive workload: a 2:1 balanced octree over a 512^3 box, uniform
    to level 3 and refined three more levels where rho > 1e-3 of the peak
    (1296 leaf sub-grids on levels 3..6, the two polytropes of the 128^3
    workload).  One step = forward + adjoint.  Returns the bench object and
    the sampled GPU outputs for the oracle check."""
    import numpy as np
    import torch

    from paper_2412_15518_amd import fmm, workloads as W
    d = W.adaptive_two_polytropes()
    lay = d["layout"]
    c0 = time.perf_counter()
    plan = fmm.Plan(lay)
    t_plan = time.perf_counter() - c0
    info = plan.info()
    N = info["n_leaf_cells"]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()    # noqa: E731
    rho, w, u = dev(d["rho"]), dev(d["w"]), dev(d["u"]).reshape(-1)
    phi = torch.empty(N, dtype=torch.float64, device="cuda")
    g = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    drho = torch.empty(N, dtype=torch.float64, device="cuda")

    def step():
        plan.forward_into(rho, phi, g)
        plan.adjoint_into(w, u, drho)

    for _ in range(3):
        step()
    kp = max(1, min(args.steps, 10))
    plan.timing_begin(2 * kp)
    for _ in range(kp):
        step()
    prof = plan.timing_end()
    phases = {k: v for k, v in prof["phases"].items() if k != "total" and v["launches"] > 0}
    k = max(5, min(args.steps, 50))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / k
    pairs = 2 * (info["p2p_pairs"] + info["m2l_pairs"])
    flops = info["flops_forward"] + info["flops_adjoint"]
    prof_ms = prof["phases"]["total"]["ms"]
    per_phase = {name: {"avg_ms": v["ms"] / v["events"], "share": v["ms"] / prof_ms} for name, v in phases.items()}
    m2l_ms = per_phase["m2l"]["avg_ms"]
    levels = np.bincount(lay.level[lay.leaf_nodes], minlength=lay.depth + 1).tolist()
    log(f"adaptive tree: {ms:.3f} ms per forward + adjoint step")
    out = {"workload": "2:1 balanced adaptive octree over a 512^3 box (h = 1): uniform to level 3 (64^3), refined "
                       "3 more levels where a cell centre has rho > 1e-3 rho_peak; two n=1.5 polytropes (rho_c "
                       "1.0/0.6, R 20/14 cells, 50 apart) + 1e-10 floor, +-1% noise; one step = forward + adjoint",
           "leaf_subgrids_per_level": levels, "n_leaf_cells": N, "n_nodes": lay.n_nodes,
           "plan_create_s": t_plan, "device_bytes": info["device_bytes"],
           "steps": k, "ms_per_step": ms, "cell_interactions_per_step": pairs,
           "cell_interactions_per_s": pairs / (ms * 1e-3),
           "fp64_flops_per_s": flops / (ms * 1e-3), "frac_fp64_peak": flops / (ms * 1e-3) / PEAK_FP64,
           "m2l_tflops": 168.0 * info["m2l_pairs"] / (m2l_ms * 1e-3) / 1e12, "phases": per_phase}
    lvl = np.repeat(lay.level[lay.leaf_nodes], 512)
    rng = np.random.default_rng(23)
    sk = np.concatenate([rng.choice(np.nonzero(lvl == l)[0], 64, replace=False) for l in np.unique(lvl)])
    gs = g.reshape(3, N)
    state = {"layout": lay, "rho": d["rho"], "sinks": sk, "phi": phi[sk].cpu().numpy(),
             "g": gs[:, sk].cpu().numpy()}
    return out, state


def bench_am(args, lay, rho_dense) -> dict:
    """The angular-momentum correction at 128^3: time per call, and the total
    torque of the forward's forces with and without the spin torques."""
    import numpy as np
    import torch

    from paper_2412_15518_amd import fmm
    plan = fmm.Plan(lay, am_correction=True)
    rho = torch.from_numpy(lay.dense_to_layout(rho_dense)).cuda()
    N = rho.numel()
    t = torch.empty((3, N), dtype=torch.float64, device="cuda")
    for _ in range(2):
        t = plan.am_correction(rho)
    k = max(3, min(args.steps, 20))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        t = plan.am_correction(rho)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / k
    _, g = plan.forward(rho)
    torch.cuda.synchronize()
    n = rho_dense.shape[-1]
    c = np.arange(n) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    X = lay.dense_to_layout(np.stack([x, y, z])).T
    m = rho.cpu().numpy()
    orb = np.cross(X, (m[None] * g.cpu().numpy()).T)
    spin = (m[None] * t.cpu().numpy()).T
    scale = float(np.abs(orb).sum())
    log(f"angular-momentum correction: {ms:.3f} ms per call")
    return {"ms_per_call": ms, "calls": k,
            "orbital_torque_rel": float(np.abs(orb.sum(0)).max() / scale),
            "with_spin_torque_rel": float(np.abs(orb.sum(0) + spin.sum(0)).max() / scale),
            "note": "spin torque per unit mass t (3 per leaf cell), FP64; |sum m (x x g)| and "
                    "|sum m (x x g + t)| over sum |m x x g|, g from the same plan's forward"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-slab", type=int, default=64,
                    help="leaf z-layers of the 128^3 grid in the CPU-oracle sample (0: skip)")
    ap.add_argument("--batch", type=int, default=1,
                    help="also time the batch of 16 independent octrees (0: skip)")
    ap.add_argument("--amr", type=int, default=1,
                    help="1: also time the adaptive-octree workload (1296 leaf sub-grids, levels 3..6)")
    ap.add_argument("--am", type=int, default=1,
                    help="1: also time the angular-momentum correction at 128^3")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before warmup, copy this many MiB device to device once: a plain copy "
                         "kernel of known traffic that calibrates HBM counter readings")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2412_15518_amd import fmm, workloads as W

    torch.cuda.set_device(0)
    log("generating the 128^3 two-polytrope workload")
    cfg = W.two_polytropes()
    lay = W.uniform_layout(cfg["L"])
    plan = fmm.Plan(lay, theta=0.4, order=3)
    info = plan.info()
    N = info["n_leaf_cells"]
    dev = lambda a: torch.from_numpy(lay.dense_to_layout(a)).cuda()   # noqa: E731
    rho, w, u = dev(cfg["rho"]), dev(cfg["w"]), dev(cfg["u"])
    phi = torch.empty(N, dtype=torch.float64, device="cuda")
    g = torch.empty((3, N), dtype=torch.float64, device="cuda")
    drho = torch.empty(N, dtype=torch.float64, device="cuda")

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.copy_mib} MiB")
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        plan.forward_into(rho, phi, g)
        plan.adjoint_into(w, u.reshape(-1), drho)
    torch.cuda.synchronize()

    # untimed pass with events around every phase: the per-phase breakdown and
    # the kernel with the largest share
    kp = max(1, min(args.steps, 10))
    plan.timing_begin(2 * kp)
    for _ in range(kp):
        plan.forward_into(rho, phi, g)
        plan.adjoint_into(w, u.reshape(-1), drho)
    prof = plan.timing_end()
    phases = {k: v for k, v in prof["phases"].items() if k != "total" and v["launches"] > 0}
    dom = max(phases, key=lambda k: phases[k]["ms"])

    # timed region: events only around that kernel's launches
    log(f"timing {args.steps} steps")
    plan.timing_begin(2 * args.steps)
    plan.timing_phases([dom])
    torch.cuda.synchronize()            # (one rank: the barrier is this synchronisation)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.forward_into(rho, phi, g)
        plan.adjoint_into(w, u.reshape(-1), drho)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = plan.timing_end()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps

    pairs_step = 2 * (info["p2p_pairs"] + info["m2l_pairs"])
    flops_step = info["flops_forward"] + info["flops_adjoint"]
    value = pairs_step * args.steps / elapsed
    fp64 = flops_step * args.steps / elapsed

    d = tim["phases"][dom]
    avg_ms = d["ms"] / d["events"]
    fl_launch = phase_flops(dom, info)
    achieved = fl_launch / (avg_ms * 1e-3) / 1e12
    traffic = read_traffic(dom)
    prof_ms = prof["phases"]["total"]["ms"]
    per_phase = {k: {"avg_ms": v["ms"] / v["events"], "share": v["ms"] / prof_ms,
                     "tflops": phase_flops(k, info) / (v["ms"] / v["events"] * 1e-3) / 1e12
                     }
                 for k, v in phases.items()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "two n=1.5 polytropes (rho_c 1.0/0.6, R 20/14 cells, 50 apart) + 1e-10 floor, "
                               "+-1% noise; uniform octree depth 4 = 128^3 cells in 4096 sub-grids of 8^3; "
                               "theta 0.4, order 3; one step = forward + adjoint",
                   "grid": 128, "depth": 4, "theta": 0.4, "order": 3,
                   "cell_interactions_per_step": pairs_step, "fp64_flop_per_step": flops_step},
        "fp64_flops_per_s": fp64,
        "frac_fp64_peak": fp64 / PEAK_FP64,
        "roofline": {"bound": "alu", "kernel": KERNEL_OF_PHASE[dom], "achieved": achieved,
                     "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s", "frac": achieved / (PEAK_FP64 / 1e12),
                     "traffic": traffic, "avg_launch_ms": avg_ms, "flop_per_launch": fl_launch,
                     "issued_flop_per_launch": fl_launch * ISSUED_PER_ALGORITHMIC.get(dom, 1.0),
                     "issued_frac": achieved * ISSUED_PER_ALGORITHMIC.get(dom, 1.0) / (PEAK_FP64 / 1e12),
                     "note": "achieved counts the algorithmic 168 FLOP per M2L pair (84 FMA of the "
                             "order-3 contraction); the kernel issues 140 (70 FMA of its traceless-reduced "
                             "form), which issued_* reports"},
        "phases": per_phase,
    }

    # the FP32 M2L (plan flag OT_FMM_M2L_FP32) on the same workload: step time,
    # M2L time and deviation from the FP64 path; the headline stays FP64
    plan32 = fmm.Plan(lay, theta=0.4, order=3, m2l_fp32=True)
    phi32 = torch.empty_like(phi)
    g32 = torch.empty_like(g)
    drho32 = torch.empty_like(drho)
    for _ in range(max(1, args.warmup)):
        plan32.forward_into(rho, phi32, g32)
        plan32.adjoint_into(w, u.reshape(-1), drho32)
    k32 = max(1, min(args.steps, 20))
    plan32.timing_begin(2 * k32)
    plan32.timing_phases(["m2l"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(k32):
        plan32.forward_into(rho, phi32, g32)
        plan32.adjoint_into(w, u.reshape(-1), drho32)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    tim32 = plan32.timing_end()
    ms32 = 1e3 * (t3 - t2) / k32
    m32 = tim32["phases"]["m2l"]["ms"] / tim32["phases"]["m2l"]["events"]

    def nw(a, b):
        return float((a - b).abs().max() / b.abs().max())

    def nwv(a, b):
        return float(((a - b) ** 2).sum(0).sqrt().max() / (b ** 2).sum(0).sqrt().max())

    out["m2l_fp32"] = {
        "ms_per_step": ms32, "speedup_step": ms_per_step / ms32,
        "m2l_avg_ms": m32, "speedup_m2l": avg_ms / m32 if dom == "m2l" else None,
        "err_vs_fp64_path": {"phi": nw(phi32, phi), "g": nwv(g32, g), "drho": nw(drho32, drho),
                             "phi_rel_l2": float((phi32 - phi).norm() / phi.norm()),
                             "g_rel_l2": float((g32 - g).norm() / g.norm()),
                             "norm": "normwise max-abs (g: per-cell Euclidean) and relative L2, whole grid"},
        "note": "M2L in FP32 with FP64 accumulation per parent offset; unpacked FP32 issues at the FP64 rate"}

    if args.batch:
        out["batch"] = bench_batch(args)
    if args.am:
        out["am_correction"] = bench_am(args, lay, cfg["rho"])
    amr_state = None
    if args.amr:
        out["amr"], amr_state = bench_amr(args)

    if args.cpu_slab > 0:
        import oracle as O
        z0 = 64 - args.cpu_slab // 2
        z1 = z0 + args.cpu_slab
        p2p, m2l = O.pair_counts(cfg["L"], 0.4, zslab=(z0, z1))
        sample_pairs = p2p + int(m2l.sum())
        log(f"CPU oracle on leaf z-slab [{z0},{z1}) with {O.threads()} threads")
        c0 = time.perf_counter()
        po, go = O.fmm(cfg["rho"], zslab=(z0, z1))
        c1 = time.perf_counter()
        do = O.fmm_adjoint(cfg["w"], cfg["u"], zslab=(z0, z1))
        c2 = time.perf_counter()
        out["cpu_baseline"] = {"value": 2 * sample_pairs / (c2 - c0), "unit": "cell-interactions/s",
                               "cores": O.threads(), "kind": "oracle",
                               "sample": f"forward + adjoint of the same 128^3 workload, sinks restricted to leaf "
                                         f"z-slab [{z0},{z1}) ({2 * sample_pairs:.4g} cell-interactions, "
                                         f"{c2 - c0:.1f} s)"}
        ph = lay.layout_to_dense(phi.cpu().numpy())[z0:z1]
        gg = lay.layout_to_dense(g.cpu().numpy())[:, z0:z1]
        dr = lay.layout_to_dense(drho.cpu().numpy())[z0:z1]
        po, go, do = po[z0:z1], go[:, z0:z1], do[z0:z1]
        out["oracle_err"] = {
            "phi": float(np.abs(ph - po).max() / np.abs(po).max()),
            "g": float(np.sqrt(((gg - go) ** 2).sum(0)).max() / np.sqrt((go ** 2).sum(0)).max()),
            "drho": float(np.abs(dr - do).max() / np.abs(do).max()),
            "norm": "normwise max-abs, over the oracle z-slab", "tolerance": 1e-12}
        ph32 = lay.layout_to_dense(phi32.cpu().numpy())[z0:z1]
        gg32 = lay.layout_to_dense(g32.cpu().numpy())[:, z0:z1]
        dr32 = lay.layout_to_dense(drho32.cpu().numpy())[z0:z1]
        out["m2l_fp32"]["err_vs_oracle_slab"] = {
            "phi": float(np.abs(ph32 - po).max() / np.abs(po).max()),
            "g": float(np.sqrt(((gg32 - go) ** 2).sum(0)).max() / np.sqrt((go ** 2).sum(0)).max()),
            "drho": float(np.abs(dr32 - do).max() / np.abs(do).max()), "tolerance": 1e-5}
        if amr_state is not None:
            st = amr_state
            c3 = time.perf_counter()
            pa, ga = O.amr_fmm_sinks(st["layout"], st["rho"], st["sinks"])
            c4 = time.perf_counter()
            out["amr"]["oracle_err"] = {
                "phi": float(np.abs(st["phi"] - pa).max() / np.abs(pa).max()),
                "g": float(np.sqrt(((st["g"] - ga) ** 2).sum(0)).max() / np.sqrt((ga ** 2).sum(0)).max()),
                "norm": f"normwise max-abs over {st['sinks'].size} sampled leaf cells, 64 per leaf level "
                        f"(oracle: {c4 - c3:.2f} s on {O.threads()} threads)", "tolerance": 1e-12}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
