"""Benchmark of the Navier-Stokes momentum RHS assembly on one MI355X.

One step = FP64 forward assembly + FP64 velocity VJP (the whole hot path:
gather, geometry, gradients, element terms, scatter-add, adjoint; the gather
scatter writes every node, so no zero-fill is needed) on the 96^3-cell
jittered, relabelled cube (5,308,416 tets, 912,673 nodes), inputs resident in
HBM in mesh order.  Prints one JSON line; defaults: 200 untimed and 200 timed
steps.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP64_PEAK_TFS = 78.6           # MI355X FP64 vector: 256 CUs x 2.4 GHz x 128 flop/cycle

# Algorithmic floating-point operations per element (add/sub/mul/div = 1,
# FMA = 2, sqrt/cbrt = 1): the element steps of the method evaluated literally
# -- Jacobian and adjugate inverse, gradients, Smagorinsky viscosity when on,
# four Gauss points, viscous term -- plus the 12 additions of the scatter, as
# the oracle's op-counting scalar type counts them (a CPU test checks these
# constants against that count).  The kernels reach the same result with
# fewer operations (the Gauss sums collapse in closed form); what they
# execute is measured with rocprofv3 VALU counters (valu_<workload>.json).
ALGORITHMIC_FLOPS = {("fwd", False): 528, ("fwd", True): 571, ("vjp", False): 827, ("vjp", True): 990}

PROFILE_DIR = os.path.join(ROOT, "profiles")


def algorithmic_bytes(ne: int, nn: int, mode: str, elem_bytes: int) -> float:
    """Bytes one launch must move with perfect nodal reuse: int32 connectivity
    once per element, every nodal array read or written once (coordinates are
    always FP64)."""
    conn = 16.0 * ne
    x = 24.0 * nn
    vec = 3 * elem_bytes * nn
    if mode == "fwd":        # x, u, p in; rhs out
        return conn + x + vec + elem_bytes * nn + vec
    return conn + x + vec + vec + vec   # x, u, adjoint in; grad out


def kernel_label(scatter: str, mode: str) -> str:
    name = {"patch_gather": "k_assemble_patch + k_gather_partials", "patch": "k_assemble_patch",
            "atomic": "k_assemble_atomic"}[scatter]
    return f"{name} ({'forward' if mode == 'fwd' else 'VJP'}, FP64)"


def source_digest() -> str:
    """Digest of the HIP sources, to tell whether stored counters are current."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_08777_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload: str, mode: str, scatter: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary of this workload, or None if there is none or the kernels changed
    since it was taken."""
    path = os.path.join(PROFILE_DIR, f"traffic_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest() or rec.get("scatter") != scatter:
        return None
    entry = rec.get("calls", {}).get(mode)
    return None if entry is None else entry.get("bytes")


def executed_flops(workload: str, mode: str):
    """FP64 flops one benchmark call executes (patch kernel and gather, every
    lane of every FP64 VALU instruction) from the committed rocprofv3 VALU
    counter record, or None if there is none or the kernels changed since."""
    path = os.path.join(PROFILE_DIR, f"valu_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_digest():
        return None
    entry = rec.get("calls", {}).get(mode)
    return None if entry is None else entry.get("fp64_flops")


def executed_rate(workload: str, mode: str, call_ms: float, ne: int):
    """The call's executed FP64 flops (VALU counters) as a rate and a fraction
    of the FP64 vector peak, or None without a current counter record."""
    fl = executed_flops(workload, mode)
    if fl is None:
        return None
    tfs = fl / (call_ms * 1e-3) / 1e12
    return {"flops_per_element": fl / ne, "achieved": tfs, "frac": tfs / FP64_PEAK_TFS}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # The GPU's clocks rise over the first ~10 ms of sustained work: 200
    # untimed steps reach the steady state, 200 timed steps take ~45 ms.
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="cube96_jit_perm")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--scatter", default="auto", choices=["auto", "atomic", "patch"])
    ap.add_argument("--patch-elems", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay of the step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also time a plain device copy of 1 GiB (HBM bandwidth and counter calibration)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library assembles on one GPU; multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2403_08777_amd import api, synth

    wl = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    m, u_np, p_np, lam_np = synth.build(wl)
    log(f"[bench] workload {wl.name}: {m.n_elems} tets, {m.n_nodes} nodes (generated in "
        f"{time.perf_counter() - t0:.1f} s)")
    coords = torch.from_numpy(m.coords).to(dev)
    conn = torch.from_numpy(m.conn).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = api.Mesh(coords, conn, renumber=True, scatter=args.scatter, patch_elems=args.patch_elems)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] mesh_create {create_ms:.1f} ms, info {mesh.info}")

    prm = api.Params(wl.rho, wl.mu, wl.cs, wl.body_force)
    ne, nn = m.n_elems, m.n_nodes

    def to_dev(a, dtype):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)

    u_user = to_dev(u_np, torch.float64)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    u = mesh.to_mesh_order(u_user)
    stop.record()
    torch.cuda.synchronize()
    reorder_ms = start.elapsed_time(stop)
    p = mesh.to_mesh_order(to_dev(p_np, torch.float64))
    lam = mesh.to_mesh_order(to_dev(lam_np, torch.float64))
    rhs = torch.empty_like(u)
    grad = torch.empty_like(u)

    def step():
        api.assemble_rhs(mesh, u, p, prm, out=rhs)
        api.assemble_rhs_vjp(mesh, u, lam, prm, out=grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")
    # timed region: exactly K steps, bracketed by synchronisation
    torch.cuda.synchronize()
    start.record()
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    ms_per_step = start.elapsed_time(stop) / args.steps
    value = ne / (ms_per_step * 1e-3)
    log(f"[bench] {args.steps} steps: {ms_per_step:.4f} ms/step (wall {wall_ms / args.steps:.4f}), "
        f"{value / 1e9:.2f} G elem/s fwd+VJP")
    # the two calls' durations inside the step: the same K steps again with
    # an event between the calls (each call's kernels and their boundary)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for e0, e1, e2 in evs:
        e0.record()
        api.assemble_rhs(mesh, u, p, prm, out=rhs)
        e1.record()
        api.assemble_rhs_vjp(mesh, u, lam, prm, out=grad)
        e2.record()
    torch.cuda.synchronize()
    in_step = {"fwd": sorted(e0.elapsed_time(e1) for e0, e1, _ in evs),
               "vjp": sorted(e1.elapsed_time(e2) for _, e1, e2 in evs)}

    # the same step captured once in a HIP graph and replayed K times (no
    # host launch overhead between the four kernels); the replay must
    # reproduce the eager outputs bit for bit (gather scatter: fixed order)
    graph = None
    if not args.no_graph:
        ref_rhs, ref_grad = rhs.clone(), grad.clone()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(rhs, ref_rhs) and torch.equal(grad, ref_grad))
        start.record()
        for _ in range(args.steps):
            g.replay()
        stop.record()
        torch.cuda.synchronize()
        g_ms = start.elapsed_time(stop) / args.steps
        graph = {"ms_per_step": g_ms, "elems_per_s": ne / (g_ms * 1e-3), "bitwise_equal_to_eager": same}
        log(f"[bench] HIP graph replay: {g_ms:.4f} ms/step, {ne / (g_ms * 1e-3) / 1e9:.2f} G elem/s "
            f"(bitwise equal to eager: {same})")
        del g

    # per-call durations of the assembly kernels alone, HIP events on the
    # launch stream; with atomic scatter, ACCUMULATE skips the zero-fill
    # kernel (the gather scatter has none)
    def kernel_ms(fn, reps):
        """(mean, median, min, max) ms of one call: the mean of calls back to
        back between one pair of events (no event between calls, as in the
        timed steps; the median over five blocks, so that one stalled block
        does not stand for the call), the others from calls timed one by one."""
        for _ in range(2):  # first launches of a kernel load its code object
            fn()
        per = max(1, reps // 5)
        blocks = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(per):
                fn()
            b.record()
            torch.cuda.synchronize()
            blocks.append(a.elapsed_time(b) / per)
        mean = float(np.median(blocks))
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        t = sorted(a.elapsed_time(b) for a, b in evs)
        return float(mean), float(np.median(t)), t[0], t[-1]

    scratch = torch.zeros_like(u)
    acc = mesh.info["scatter"] != "patch_gather"
    fwd_k = kernel_ms(lambda: api.assemble_rhs(mesh, u, p, prm, out=scratch, accumulate=acc), args.kernel_reps)
    vjp_k = kernel_ms(lambda: api.assemble_rhs_vjp(mesh, u, lam, prm, out=scratch, accumulate=acc),
                      args.kernel_reps)
    fill_k = kernel_ms(lambda: scratch.zero_(), args.kernel_reps)
    # mean/median/min/max: the call inside the timed step; alone_*: the same
    # call repeated on its own (FP64-dense VJPs back to back run slower)
    kernels = {k: {"mean_ms": float(np.mean(t)), "median_ms": float(np.median(t)), "min_ms": t[0], "max_ms": t[-1],
                   "alone_mean_ms": ka[0], "alone_median_ms": ka[1],
                   "alg_bytes": algorithmic_bytes(ne, nn, k, 8)}
               for k, t, ka in (("fwd", in_step["fwd"], fwd_k), ("vjp", in_step["vjp"], vjp_k))}
    kernels["zero_fill_equiv"] = {"mean_ms": fill_k[0]}
    eddy = wl.cs > 0
    for k in ("fwd", "vjp"):
        kk = kernels[k]
        kk["elems_per_s"] = ne / (kk["mean_ms"] * 1e-3)
        kk["alg_GBs"] = kk["alg_bytes"] / (kk["mean_ms"] * 1e-3) / 1e9
        kk["alg_flops"] = ALGORITHMIC_FLOPS[(k, eddy)] * ne
        kk["alg_TFs"] = kk["alg_flops"] / (kk["mean_ms"] * 1e-3) / 1e12
        kk["hbm_frac"] = kk["alg_GBs"] / HBM_PEAK_GBS
        kk["fp64_frac"] = kk["alg_TFs"] / FP64_PEAK_TFS
        # measured HBM bytes of the call (committed counter record), when current
        tb = measured_traffic(wl.name, k, mesh.info["scatter"])
        kk["traffic_GBs"] = tb / (kk["mean_ms"] * 1e-3) / 1e9 if tb else None
    dom = max(("fwd", "vjp"), key=lambda k: kernels[k]["mean_ms"])
    kd = kernels[dom]
    log(f"[bench] calls in the step: fwd {kernels['fwd']['mean_ms']:.4f} ms, vjp {kernels['vjp']['mean_ms']:.4f} ms "
        f"(alone: {fwd_k[0]:.4f}, {vjp_k[0]:.4f}; dominant: {dom})")

    forms = {"fp64_fwd_elems_per_s": kernels["fwd"]["elems_per_s"]}
    # mixed precision on the same mesh: fields FP32, geometry FP64
    if not args.no_mixed:
        u32, p32, l32 = u.float(), p.float(), lam.float()
        r32, g32 = torch.empty_like(u32), torch.empty_like(u32)

        def step32():
            api.assemble_rhs(mesh, u32, p32, prm, out=r32)
            api.assemble_rhs_vjp(mesh, u32, l32, prm, out=g32)

        for _ in range(args.warmup):
            step32()
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            step32()
        stop.record()
        torch.cuda.synchronize()
        ms32 = start.elapsed_time(stop) / args.steps
        f32 = kernel_ms(lambda: api.assemble_rhs(mesh, u32, p32, prm, out=r32), args.kernel_reps)
        forms["mixed_fwd_vjp_elems_per_s"] = ne / (ms32 * 1e-3)
        forms["mixed_fwd_elems_per_s"] = ne / (f32[0] * 1e-3)

    # the selectable physics (eddy-viscosity models, convective forms) and the
    # other derivative products, FP64 on the same mesh: per-call kernel times
    # and the resulting rate of one forward + VJP pair
    variants = {}
    pr_g = torch.empty(nn, dtype=torch.float64, device=dev)
    du = torch.randn_like(u)
    dpr = torch.randn_like(p)
    for tag, cs, model, conv in (("smagorinsky", 0.1, "smagorinsky", "advective"),
                                 ("vreman", 0.1, "vreman", "advective"),
                                 ("divergence", wl.cs, "smagorinsky", "divergence"),
                                 ("skew", wl.cs, "smagorinsky", "skew"),
                                 ("rotational", wl.cs, "smagorinsky", "rotational"),
                                 ("emac", wl.cs, "smagorinsky", "emac")):
        vp = api.Params(wl.rho, wl.mu, cs, wl.body_force, model, conv)
        # means of calls back to back, as for the benchmark calls
        tf = kernel_ms(lambda: api.assemble_rhs(mesh, u, p, vp, out=scratch, accumulate=acc), args.kernel_reps)[0]
        tv = kernel_ms(lambda: api.assemble_rhs_vjp(mesh, u, lam, vp, out=scratch, accumulate=acc),
                       args.kernel_reps)[0]
        variants[tag] = {"eddy_model": model, "smagorinsky_cs": cs, "convective_form": conv, "fwd_ms": tf,
                         "vjp_ms": tv, "fwd_vjp_elems_per_s": ne / ((tf + tv) * 1e-3)}
    tj = kernel_ms(lambda: api.assemble_rhs_jvp(mesh, u, du, dpr, prm, out=scratch, accumulate=acc),
                   args.kernel_reps)[0]
    tp = kernel_ms(lambda: api.assemble_rhs_vjp_p(mesh, lam, prm, out=pr_g, accumulate=acc), args.kernel_reps)[0]
    variants["jvp"] = {"ms": tj, "elems_per_s": ne / (tj * 1e-3)}
    variants["vjp_p"] = {"ms": tp, "elems_per_s": ne / (tp * 1e-3)}

    # the same forward + VJP through torch.autograd (NSAssembleRHS): output
    # allocation and autograd bookkeeping included
    u_req = u.detach().clone().requires_grad_(True)

    def autograd_step():
        u_req.grad = None
        api.NSAssembleRHS.apply(u_req, p, mesh, prm).backward(lam)

    ta = kernel_ms(autograd_step, args.kernel_reps)[0]
    variants["autograd_fwd_bwd"] = {"ms": ta, "elems_per_s": ne / (ta * 1e-3)}
    # explicit momentum stage u + dt R / (rho V^L) with a boundary Dirichlet
    # mask; with the gather scatter the update is fused into the gather kernel
    bnd = np.any((m.coords < 1e-12) | (m.coords > 1 - 1e-12), axis=1)
    mask = mesh.to_mesh_order(to_dev(np.where(bnd, 7.0, 0.0), torch.float64)).to(torch.uint8)
    tu = kernel_ms(lambda: api.explicit_update(mesh, u, p, prm, 1e-3, mask, out=scratch), args.kernel_reps)[0]
    variants["explicit_update"] = {"ms": tu, "elems_per_s": ne / (tu * 1e-3),
                                   "fused": mesh.info["scatter"] == "patch_gather",
                                   "vs_forward_ms": tu - kernels["fwd"]["mean_ms"]}
    log("[bench] variants (fwd+vjp G elem/s): " + ", ".join(
        f"{k} {v['fwd_vjp_elems_per_s'] / 1e9:.2f}" for k, v in variants.items() if "fwd_vjp_elems_per_s" in v)
        + f"; jvp {tj * 1e3:.1f} us, vjp_p {tp * 1e3:.1f} us, explicit update {tu * 1e3:.1f} us, "
        f"autograd forward + backward {ta * 1e3:.1f} us")

    result = {
        "metric": "elements/s (FP64 forward + velocity VJP assembly)",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.n}^3-cell unit cube, 6 tets/cell, jitter={wl.jitter}, "
                               f"relabelled={wl.permute}", "n_elems": ne, "n_nodes": nn, "mu": wl.mu,
                   "smagorinsky_cs": wl.cs, "scatter": mesh.info["scatter"],
                   "patch_elems": mesh.info["patch_elems"]},
        "roofline": {"bound": "alu", "kernel": kernel_label(mesh.info["scatter"], dom),
                     "achieved": kd["alg_TFs"], "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": kd["alg_TFs"] / FP64_PEAK_TFS,
                     "traffic": measured_traffic(wl.name, dom, mesh.info["scatter"]),
                     "flops_per_element": ALGORITHMIC_FLOPS[(dom, eddy)], "elements_per_launch": ne,
                     "executed": executed_rate(wl.name, dom, kd["mean_ms"], ne)},
        "kernels": kernels,
        "forms": forms,
        "variants": variants,
        "graph_replay": graph,
        "setup": {"mesh_create_ms": create_ms, "to_mesh_order_ms_per_vector_field": reorder_ms,
                  "device": torch.cuda.get_device_name(dev), "hip": getattr(torch.version, "hip", None)},
    }

    # attainable HBM bandwidth: the library's Scale kernel (b = s a) over two
    # 1 GiB FP64 arrays, far beyond the last-level cache; with the FP64 peak it
    # gives the machine balance, as the paper does with its measured Scale rate
    sc_a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    sc_b = torch.empty_like(sc_a)
    sk = kernel_ms(lambda: api.stream_scale(sc_a, 3.0, out=sc_b), 20)
    sc_bytes = 16 * sc_a.numel()
    sc_gbs = sc_bytes / (sk[0] * 1e-3) / 1e9
    result["hbm_scale"] = {"bytes_per_call": sc_bytes, "mean_ms": sk[0], "median_ms": sk[1], "GBs": sc_gbs,
                           "frac_of_peak": sc_gbs / HBM_PEAK_GBS,
                           "machine_balance_flop_per_byte": FP64_PEAK_TFS * 1e3 / sc_gbs}
    log(f"[bench] Scale kernel over 2 x 1 GiB: {sk[0]:.3f} ms, {sc_gbs:.0f} GB/s "
        f"({sc_gbs / HBM_PEAK_GBS:.2f} of peak; machine balance {FP64_PEAK_TFS * 1e3 / sc_gbs:.1f} flop/B)")
    # each call's bandwidth also as a fraction of what the Scale kernel draws
    for k in ("fwd", "vjp"):
        kk = kernels[k]
        kk["alg_frac_of_scale"] = kk["alg_GBs"] / sc_gbs
        kk["traffic_frac_of_scale"] = kk["traffic_GBs"] / sc_gbs if kk["traffic_GBs"] else None
    del sc_a, sc_b

    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        cp = kernel_ms(lambda: b.copy_(a), 5)
        result["copy_calibration"] = {"bytes_read": nbytes, "bytes_written": nbytes, "mean_ms": cp[0],
                                      "GBs_read_plus_write": 2 * nbytes / (cp[0] * 1e-3) / 1e9}
        log(f"[bench] copy of 1 GiB: {cp[0]:.3f} ms, {2 * nbytes / (cp[0] * 1e-3) / 1e9:.0f} GB/s (read+write)")
        del a, b

    if not args.no_cpu_baseline:
        import oracle

        oprm = oracle.Params(wl.rho, wl.mu, wl.cs, wl.body_force)
        threads = oracle.default_threads()
        # passes over the full mesh until about 10 s of host work (at least 3)
        times = []
        while len(times) < 3 or (sum(times) < 10.0 and len(times) < 50):
            t0 = time.perf_counter()
            r_ref = oracle.rhs(m.coords, m.conn, u_np, p_np, oprm, nthreads=threads)
            g_ref = oracle.vjp(m.coords, m.conn, u_np, lam_np, oprm, nthreads=threads)
            times.append(time.perf_counter() - t0)
        t_cpu = float(np.median(times))
        result["cpu_baseline"] = {"value": ne / t_cpu, "unit": "elements/s", "cores": threads, "kind": "oracle",
                                  "sample": f"FP64 forward + VJP of the C oracle over the full {wl.n}^3 mesh "
                                            f"({ne} tets), median of {len(times)} passes "
                                            f"({sum(times):.1f} s of host work): {t_cpu:.2f} s wall each"}
        # one host thread on the first eighth of the elements (the paper reports 1 core beside the node)
        sub = np.ascontiguousarray(m.conn[: max(1, ne // 8)])
        t1 = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.rhs(m.coords, sub, u_np, p_np, oprm, nthreads=1)
            oracle.vjp(m.coords, sub, u_np, lam_np, oprm, nthreads=1)
            t1.append(time.perf_counter() - t0)
        result["cpu_baseline"]["one_thread"] = {
            "value": sub.shape[0] / float(np.median(t1)), "unit": "elements/s", "cores": 1,
            "sample": f"FP64 forward + VJP of the C oracle on the first {sub.shape[0]} tets, median of 3 passes"}
        # accuracy of the timed outputs against the oracle (user order)
        err = {"fp64_rhs": oracle.rel_l2(mesh.from_mesh_order(rhs).cpu().numpy(), r_ref),
               "fp64_grad": oracle.rel_l2(mesh.from_mesh_order(grad).cpu().numpy(), g_ref)}
        if not args.no_mixed:
            err["mixed_rhs"] = oracle.rel_l2(mesh.from_mesh_order(r32).double().cpu().numpy(), r_ref)
            err["mixed_grad"] = oracle.rel_l2(mesh.from_mesh_order(g32).double().cpu().numpy(), g_ref)
        result["rel_l2_vs_oracle"] = err
        log(f"[bench] oracle {t_cpu:.2f} s on {threads} threads; errors {err}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
