"""Benchmark of the Navier-Stokes momentum RHS assembly on one MI355X.

Headline step (``value``): FP64 forward assembly + FP64 velocity VJP (the whole
hot path: gather, geometry, gradients, element terms, scatter-add, adjoint) on
the 96^3-cell jittered, relabelled cube (5,308,416 tets, 912,673 nodes),
inputs resident in HBM in mesh order.  After W untimed steps the K-step
timed region is repeated as back-to-back blocks of exactly K steps (at least
five, and at least 2000 steps in all) and ``ms_per_step`` is the median block;
the first block is reported beside it.

``configs`` carries one record per workload of the method's measurement plan:
  C1  16^3 cube, natural ids, FP64 forward
  C2  96^3 cube, relabelled, FP64 forward
  C3  160^3 cube, jittered, relabelled, Smagorinsky C_s = 0.1, FP64 forward
  C4  96^3 cube, jittered, relabelled, FP64 forward + VJP (the headline)
  C5  the C3 mesh, mixed precision forward + VJP
each with elements/s (median block), each kernel's duration from HIP events
recorded at the kernels' own start and end (nsasm_set_kernel_events), the
roofline of the dominant kernel, the relative L2 error against the FP64
oracle over the whole mesh and the oracle's own rate on the host's threads
(and on one thread for C1 and C2).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--configs C1,C2,...]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import dataclass

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
FP64_PEAK_TFS = 78.6           # MI355X FP64 vector: 256 CUs x 2.4 GHz x 128 flop/cycle
FP32_PEAK_TFS = 157.3          # MI355X FP32 vector (vendor; needs packed FP32 instructions)
CUS = 256                      # compute units (one LDS each)
SIMDS = CUS * 4                # 4 SIMDs per compute unit
CLOCK_HZ = 2.4e9               # peak engine clock
VALU_CYCLES = 4                # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles

# Algorithmic floating-point operations per element (add/sub/mul/div = 1,
# FMA = 2, sqrt/cbrt = 1): the element steps of the method evaluated literally
# -- Jacobian and adjugate inverse, gradients, Smagorinsky viscosity when on,
# four Gauss points, viscous term -- plus the 12 additions of the scatter, as
# the oracle's op-counting scalar type counts them (a CPU test checks these
# constants against that count).  The kernels reach the same result with
# fewer operations (the Gauss sums collapse in closed form); what they
# execute is measured with rocprofv3 VALU counters (counters_<workload>.json).
ALGORITHMIC_FLOPS = {("fwd", False): 528, ("fwd", True): 571, ("vjp", False): 827, ("vjp", True): 990}

PROFILE_DIR = os.path.join(ROOT, "profiles")
PHASE_WARM_MS = 50.0           # untimed GPU work before the per-kernel timing
MIN_TIMED_STEPS = 2000         # the timed blocks cover at least this many steps (the clocks
                               # take tens of milliseconds to settle; short blocks need many)


@dataclass(frozen=True)
class Config:
    """One workload of the measurement plan: mesh recipe, precision, calls."""

    name: str
    workload: str
    precision: str           # "fp64" or "mixed"
    calls: tuple             # ("fwd",) or ("fwd", "vjp")
    one_thread: bool = False  # also time the oracle on one host thread

    @property
    def form(self) -> str:
        return "+".join(self.calls)


CONFIGS = {
    "C1": Config("C1", "cube16", "fp64", ("fwd",), one_thread=True),
    "C2": Config("C2", "cube96_perm", "fp64", ("fwd",), one_thread=True),
    "C3": Config("C3", "cube160_jit_perm_smag", "fp64", ("fwd",)),
    "C4": Config("C4", "cube96_jit_perm", "fp64", ("fwd", "vjp")),
    "C5": Config("C5", "cube160_jit_perm_smag", "mixed", ("fwd", "vjp")),
}
HEADLINE = "C4"


def algorithmic_bytes(ne: int, nn: int, mode: str, elem_bytes: int) -> float:
    """Bytes one call must move with perfect nodal reuse: int32 connectivity
    once per element, every nodal array read or written once (coordinates are
    always FP64)."""
    conn = 16.0 * ne
    x = 24.0 * nn
    vec = 3 * elem_bytes * nn
    if mode == "fwd":        # x, u, p in; rhs out
        return conn + x + vec + elem_bytes * nn + vec
    return conn + x + vec + vec + vec   # x, u, adjoint in; grad out


def kernel_names(precision: str, eddy: bool, mode: str) -> tuple:
    """(element kernel, gather kernel) of a default-physics call on a
    gather-scatter mesh, as rocprofv3 and the compiler name them."""
    t = "double" if precision == "fp64" else "float"
    m = {"fwd": 0, "vjp": 1}[mode]
    return (f"k_assemble_patch<{t}, {1 if eddy else 0}, 0, {m}, true>", f"k_gather_partials<{t}, 3>")


def source_digest() -> str:
    """Digest of the HIP sources, to tell whether stored records are current."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_08777_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def _record(path: str):
    """A committed JSON record, or None if missing, unreadable or taken with
    other HIP sources than the current ones."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_sha256") == source_digest() else None


def counter_record(workload: str):
    """Per-kernel rocprofv3 counters of a workload (HBM bytes from FETCH_SIZE /
    WRITE_SIZE scaled by a plain copy, SQ instruction and LDS counters, L2 hits)
    or None when there is no current record."""
    rec = _record(os.path.join(PROFILE_DIR, f"counters_{workload}.json"))
    return None if rec is None else rec.get("kernels")


def resource_record():
    """Per-kernel VGPRs, scratch and LDS from the compiler's resource remarks
    (profiles/resources.json), or None when not current."""
    rec = _record(os.path.join(PROFILE_DIR, "resources.json"))
    return None if rec is None else rec.get("kernels")


def kernel_evidence(ctr: dict | None, kernel: str, ms: float, scale_gbs: float | None):
    """Measured figures of one kernel from its counter entry and its live
    duration: HBM bytes and rate, executed FP64/FP32 flops and rate, how
    busy the vector ALUs and the LDS were, the LDS bank-conflict share and
    the L2 hit rate.  None without a current counter record.  Both busy
    fractions are taken at the peak engine clock: cycles counted over cycles
    available at 2.4 GHz (a lower clock under load would make the true
    fractions larger).
    SQ_LDS_IDX_ACTIVE counts the cycles a compute unit's LDS spends on indexed
    operations (its bank-conflict cycles included), summed over all units."""
    if not ctr or kernel not in ctr:
        return None
    k = ctr[kernel]
    sec = ms * 1e-3
    pw = k.get("per_wave", {})
    waves = k.get("waves", 0.0)
    out = {"hbm_bytes": k.get("hbm_bytes"), "waves": waves}
    if out["hbm_bytes"]:
        out["hbm_GBs"] = out["hbm_bytes"] / sec / 1e9
        out["hbm_frac_of_peak"] = out["hbm_GBs"] / HBM_PEAK_GBS
        out["hbm_frac_of_scale"] = out["hbm_GBs"] / scale_gbs if scale_gbs else None
    f64, f32 = k.get("f64_flops"), k.get("f32_flops")
    if f64 is not None:
        out["executed_fp64_TFs"] = f64 / sec / 1e12
        out["executed_fp32_TFs"] = (f32 or 0.0) / sec / 1e12
        # issue-limited fraction: FP32 without packed math issues at the FP64 rate
        out["executed_frac_of_valu_issue"] = (f64 + (f32 or 0.0)) / sec / 1e12 / FP64_PEAK_TFS
    if "SQ_INSTS_VALU" in pw and waves:
        out["valu_busy"] = pw["SQ_INSTS_VALU"] * waves * VALU_CYCLES / (SIMDS * CLOCK_HZ * sec)
    if pw.get("SQ_LDS_IDX_ACTIVE"):
        out["lds_conflict_share"] = pw.get("SQ_LDS_BANK_CONFLICT", 0.0) / pw["SQ_LDS_IDX_ACTIVE"]
        if waves:
            out["lds_busy"] = pw["SQ_LDS_IDX_ACTIVE"] * waves / (CUS * CLOCK_HZ * sec)
        out["lds_bank_conflict_cycles_per_wave"] = pw.get("SQ_LDS_BANK_CONFLICT")
    if k.get("l2_hit_rate") is not None:
        out["l2_hit_rate"] = k["l2_hit_rate"]
    return out


def limiter(ev: dict | None) -> tuple:
    """(bound, verdict) from the measured evidence of the dominant kernel:
    the roof it is nearest to (VALU issue or HBM, against the Scale kernel's
    attainable bandwidth), and whether it, or the LDS, actually presses on
    its limit."""
    if not ev or "valu_busy" not in ev or ev.get("hbm_frac_of_scale") is None:
        return "alu", "no current counter record: bound by algorithmic intensity only"
    busy, hbm = ev["valu_busy"], ev["hbm_frac_of_scale"]
    bound = "alu" if busy >= hbm else "hbm"
    if ev.get("waves") and ev["waves"] < SIMDS:
        return bound, (f"latency: {ev['waves']:.0f} waves cannot fill the {SIMDS} SIMDs (VALU busy {busy:.2f}, "
                       f"HBM {hbm:.2f} of the Scale bandwidth)")
    near = max(busy, hbm)
    if near >= 0.8:
        return bound, f"{'VALU issue' if bound == 'alu' else 'HBM bandwidth'} ({near:.2f} of it)"
    if ev.get("lds_busy") is not None and ev["lds_busy"] >= 0.8:
        return bound, (f"LDS throughput ({ev['lds_busy']:.2f} of it); VALU busy {busy:.2f}, "
                       f"HBM {hbm:.2f} of the Scale bandwidth")
    units = [("VALU", busy), ("HBM", hbm)]
    if ev.get("lds_busy") is not None:
        units.append(("LDS", ev["lds_busy"]))
    top, top_frac = max(units, key=lambda u: u[1])
    cs = ev.get("lds_conflict_share")
    lds = f"LDS busy {ev['lds_busy']:.2f}" if ev.get("lds_busy") is not None else "LDS busy unmeasured"
    if cs is not None:
        lds += f" (bank-conflict share {cs:.2f})"
    return bound, (f"neither roof: {lds}, VALU busy {busy:.2f}, HBM {hbm:.2f} of the Scale bandwidth; "
                   f"the busiest is {top} at {top_frac:.2f} and none is saturated: each workgroup's "
                   "dependent loads, LDS phases and arithmetic, separated by barriers, overlap only in part")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--configs", default="C1,C2,C3,C4,C5",
                    help="comma-separated subset of C1..C5 (C4 is always timed: it is the headline)")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the physics variants, the HIP-graph replay and the autograd timing")
    ap.add_argument("--scatter", default="auto", choices=["auto", "atomic", "patch"])
    ap.add_argument("--patch-elems", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also time a plain device copy of 1 GiB (HBM bandwidth and counter calibration)")
    ap.add_argument("--blocks", type=int, default=0,
                    help="timed blocks of K steps (0: at least five and at least %d steps in all)" % MIN_TIMED_STEPS)
    ap.add_argument("--unstructured", type=int, default=0, metavar="POINTS",
                    help="also time FP64 and mixed forward + VJP on the Delaunay mesh of POINTS seeded "
                         "uniform points (scipy; 1000000 points give 6.7 M tetrahedra)")
    ap.add_argument("--profile-run", action="store_true",
                    help="for profiler passes: only the listed configs, each timed briefly, no headline, "
                         "extras or oracle; prints one short JSON line")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Loaded:
    """A workload on the GPU: host arrays (user order), the mesh, and its
    fields in mesh order per precision (created on first use)."""

    def __init__(self, name, args, torch, api, synth):
        self.torch, self.api = torch, api
        self.wl = synth.WORKLOADS[name]
        t0 = time.perf_counter()
        self.m, self.u, self.p, self.lam = synth.build(self.wl)
        gen_s = time.perf_counter() - t0
        self.dev = torch.device("cuda:0")
        coords = torch.from_numpy(self.m.coords).to(self.dev)
        conn = torch.from_numpy(self.m.conn).to(self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.mesh = api.Mesh(coords, conn, renumber=True, scatter=args.scatter, patch_elems=args.patch_elems)
        torch.cuda.synchronize()
        self.create_ms = (time.perf_counter() - t0) * 1e3
        del coords, conn
        self.ne, self.nn = self.m.n_elems, self.m.n_nodes
        self.prm = api.Params(self.wl.rho, self.wl.mu, self.wl.cs, self.wl.body_force)
        self._fields = {}
        log(f"[bench] workload {name}: {self.ne} tets, {self.nn} nodes (generated in {gen_s:.1f} s), "
            f"mesh_create {self.create_ms:.1f} ms, info {self.mesh.info}")

    def fields(self, precision):
        if precision not in self._fields:
            torch = self.torch
            dt = torch.float64 if precision == "fp64" else torch.float32
            t = lambda a: self.mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(self.dev, dt))
            u, p, lam = t(self.u), t(self.p), t(self.lam)
            self._fields[precision] = (u, p, lam, torch.empty_like(u), torch.empty_like(u))
        return self._fields[precision]

    def calls(self, cfg: Config):
        api = self.api
        u, p, lam, rhs, grad = self.fields(cfg.precision)
        fns = {"fwd": lambda: api.assemble_rhs(self.mesh, u, p, self.prm, out=rhs),
               "vjp": lambda: api.assemble_rhs_vjp(self.mesh, u, lam, self.prm, out=grad)}
        return [(c, fns[c]) for c in cfg.calls]

    def close(self):
        self._fields.clear()
        self.mesh.close()


def time_blocks(torch, step, k: int, w: int, nblocks: int = 0) -> dict:
    """W untimed steps, then back-to-back blocks of exactly K steps between
    HIP events on the launch stream (by default at least five blocks and
    MIN_TIMED_STEPS steps), bracketed by device synchronisation.  Per-step
    times of every block; the median block is the figure, the first block is
    reported."""
    for _ in range(w):
        step()
    torch.cuda.synchronize()
    if nblocks <= 0:
        nblocks = max(5, math.ceil(MIN_TIMED_STEPS / k))
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(nblocks + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    marks[0].record()
    for b in range(nblocks):
        for _ in range(k):
            step()
        marks[b + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_wall) * 1e3 / (nblocks * k)
    per = [marks[b].elapsed_time(marks[b + 1]) / k for b in range(nblocks)]
    return {"median_ms": float(np.median(per)), "first_block_ms": per[0], "min_ms": min(per),
            "max_ms": max(per), "blocks": nblocks, "steps_per_block": k, "wall_ms": wall}


def time_phases(torch, api, calls, k: int, step_ms: float = 0.0) -> dict:
    """Each call's two kernels timed live inside a replica of the step,
    repeated max(K, 100) times right after untimed steps that keep the GPU
    busy for about 50 ms (at least 20; step_ms is the measured step time), with
    no synchronisation in between, so that the clocks are back where the timed
    blocks had them: nsasm_set_kernel_events has the library launch the element
    kernel and the gather kernel with HIP start/stop events that are recorded
    at the kernel's own start and end on the launch stream.  Mean and median
    duration of each kernel over the repetitions."""
    n = len(calls)
    reps = max(k, 100)
    rows = [[torch.cuda.Event(enable_timing=True) for _ in range(4 * n)] for _ in range(reps)]
    for row in rows:          # HIP events are created on their first record
        for e in row:
            e.record()
    torch.cuda.synchronize()
    warm = max(20, math.ceil(PHASE_WARM_MS / step_ms)) if step_ms > 0 else 20
    for _ in range(warm):
        for _, fn in calls:
            fn()
    for row in rows:
        for c, (_, fn) in enumerate(calls):
            api.set_kernel_events(*row[4 * c:4 * c + 4])
            fn()
    torch.cuda.synchronize()
    out = {}
    for c, (name, _) in enumerate(calls):
        el = [row[4 * c].elapsed_time(row[4 * c + 1]) for row in rows]
        ga = [row[4 * c + 2].elapsed_time(row[4 * c + 3]) for row in rows]
        out[name] = {"element_kernel_ms": float(np.mean(el)), "element_kernel_median_ms": float(np.median(el)),
                     "gather_kernel_ms": float(np.mean(ga)), "gather_kernel_median_ms": float(np.median(ga)),
                     "call_ms": float(np.mean(el) + np.mean(ga)),
                     "call_median_ms": float(np.median(el) + np.median(ga)), "repetitions": reps}
    return out


def roofline(cfg: Config, ld: Loaded, phases: dict, scale_gbs, ctr, res) -> dict:
    """Roofline of the config's dominant kernel (the longest element kernel of
    its calls): algorithmic flops per launch over its live duration against the
    vector peak of its precision, the call's algorithmic bytes over the call's
    duration against HBM, and the measured evidence of what limits it."""
    eddy = ld.wl.cs > 0
    mode = max(cfg.calls, key=lambda c: phases[c]["element_kernel_ms"])
    ph = phases[mode]
    kname, gname = kernel_names(cfg.precision, eddy, mode)
    kms, cms = ph["element_kernel_ms"], ph["call_ms"]
    fl = ALGORITHMIC_FLOPS[(mode, eddy)] * ld.ne
    peak = FP64_PEAK_TFS if cfg.precision == "fp64" else FP32_PEAK_TFS
    achieved = fl / (kms * 1e-3) / 1e12
    eb = 8 if cfg.precision == "fp64" else 4
    ab = algorithmic_bytes(ld.ne, ld.nn, mode, eb)
    ev = kernel_evidence(ctr, kname, kms, scale_gbs)
    bound, verdict = limiter(ev)
    out = {"bound": bound, "kernel": f"{kname} ({mode}, {cfg.precision})", "achieved": achieved, "peak": peak,
           "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": ev.get("hbm_bytes") if ev else None,
           "flops_per_element": ALGORITHMIC_FLOPS[(mode, eddy)], "elements_per_launch": ld.ne,
           "kernel_ms": kms,
           "call": {"kernels": [kname, gname], "ms": cms, "achieved_TFs": fl / (cms * 1e-3) / 1e12,
                    "frac": fl / (cms * 1e-3) / 1e12 / peak,
                    "alg_bytes": ab, "alg_GBs": ab / (cms * 1e-3) / 1e9,
                    "hbm_frac": ab / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "hbm_frac_of_scale": ab / (cms * 1e-3) / 1e9 / scale_gbs if scale_gbs else None},
           "limiter": verdict, "evidence": ev}
    if cfg.precision == "mixed":
        # without packed FP32 (disabled on this platform) FP32 issues at the FP64 rate
        out["frac_of_unpacked_fp32"] = achieved / FP64_PEAK_TFS
    if res:
        out["resources"] = {k: res.get(k) for k in (kname, gname)}
    return out


def oracle_leg(cfg: Config, ld: Loaded, budget_s: float, one_thread: bool):
    """The FP64 oracle over the whole mesh on the host's threads: its outputs
    (for the error of the GPU results) and its rate, as many passes as fit in
    about budget_s of host work (at least one); on one thread too when asked."""
    import oracle

    wl = ld.wl
    oprm = oracle.Params(wl.rho, wl.mu, wl.cs, wl.body_force)
    threads = oracle.default_threads()

    def run(nthreads):
        r = oracle.rhs(ld.m.coords, ld.m.conn, ld.u, ld.p, oprm, nthreads=nthreads)
        g = oracle.vjp(ld.m.coords, ld.m.conn, ld.u, ld.lam, oprm, nthreads=nthreads) if "vjp" in cfg.calls else None
        return r, g

    times, out = [], None
    while not times or (sum(times) < budget_s and len(times) < 50):
        t0 = time.perf_counter()
        out = run(threads)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    base = {"value": ld.ne / t, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 {cfg.form} of the C oracle over the whole {wl.name} mesh ({ld.ne} tets), "
                      f"median of {len(times)} passes of {t:.3f} s"}
    if one_thread:
        t1 = []
        while not t1 or (sum(t1) < budget_s and len(t1) < 5):
            t0 = time.perf_counter()
            run(1)
            t1.append(time.perf_counter() - t0)
        base["one_thread"] = {"value": ld.ne / float(np.median(t1)), "unit": "elements/s", "cores": 1,
                              "sample": f"the same on one thread, median of {len(t1)} passes"}
    return out, base


def measure_config(cfg: Config, ld: Loaded, args, torch, api, scale_gbs, res, blocks=None):
    """One config's record: median-block rate, kernel durations, roofline,
    error against the oracle and the oracle's rate."""
    calls = ld.calls(cfg)

    def step():
        for _, fn in calls:
            fn()

    if blocks is None:
        blocks = time_blocks(torch, step, args.steps, args.warmup, args.blocks)
    phases = time_phases(torch, api, calls, args.steps, blocks["median_ms"])
    ctr = counter_record(ld.wl.name)
    rec = {"workload": ld.wl.name, "n_elems": ld.ne, "n_nodes": ld.nn, "precision": cfg.precision,
           "form": cfg.form, "mu": ld.wl.mu, "smagorinsky_cs": ld.wl.cs, "mesh_create_ms": ld.create_ms,
           "elements_per_s": ld.ne / (blocks["median_ms"] * 1e-3), "ms_per_step": blocks,
           "kernels": phases, "roofline": roofline(cfg, ld, phases, scale_gbs, ctr, res)}
    if "fwd" in phases and len(cfg.calls) > 1:
        rec["fwd_elements_per_s"] = ld.ne / (phases["fwd"]["call_ms"] * 1e-3)
    log(f"[bench] {cfg.name} {ld.wl.name} {cfg.precision} {cfg.form}: {blocks['median_ms'] * 1e3:.1f} us/step "
        f"(first block {blocks['first_block_ms'] * 1e3:.1f}), {rec['elements_per_s'] / 1e9:.2f} G elem/s; "
        + ", ".join(f"{c}: {v['element_kernel_ms'] * 1e3:.1f} + {v['gather_kernel_ms'] * 1e3:.1f} us"
                    for c, v in phases.items())
        + f"; dominant frac {rec['roofline']['frac']:.3f}")
    if not args.no_cpu_baseline:
        import oracle

        u, p, lam, rhs, grad = ld.fields(cfg.precision)
        budget = 8.0 if cfg.name == HEADLINE else 3.0
        (r_ref, g_ref), base = oracle_leg(cfg, ld, budget, cfg.one_thread)
        back = lambda t: ld.mesh.from_mesh_order(t).double().cpu().numpy()
        # the outputs of the last timed call of each kind
        err = {"rhs": oracle.rel_l2(back(rhs), r_ref)}
        rd = back(rhs) - r_ref
        err["rhs_max_node"] = float(np.max(np.abs(rd)) / np.max(np.abs(r_ref)))
        if g_ref is not None:
            gd = back(grad)
            err["grad"] = oracle.rel_l2(gd, g_ref)
            err["grad_max_node"] = float(np.max(np.abs(gd - g_ref)) / np.max(np.abs(g_ref)))
        rec["rel_l2_vs_oracle"] = err
        rec["cpu_baseline"] = base
        log(f"[bench] {cfg.name} oracle {base['value'] / 1e6:.2f} M elem/s on {base['cores']} threads; "
            f"errors {err}")
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library assembles on one GPU; multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)
    names = [c.strip() for c in args.configs.split(",") if c.strip()]
    for c in names:
        if c not in CONFIGS:
            print(f"unknown config {c}; choose from {', '.join(CONFIGS)}", file=sys.stderr)
            sys.exit(2)

    import torch

    from paper_2403_08777_amd import api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    res = resource_record()

    # attainable HBM bandwidth first (a property of the machine): the library's
    # Scale kernel (b = s a) over two 1 GiB FP64 arrays, far beyond the
    # last-level cache; with the FP64 peak it gives the machine balance, as
    # the paper does with its measured Scale rate
    sc_a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    sc_b = torch.empty_like(sc_a)
    for _ in range(3):
        api.stream_scale(sc_a, 3.0, out=sc_b)
    sk = time_blocks(torch, lambda: api.stream_scale(sc_a, 3.0, out=sc_b), 4, 2, 5 if args.profile_run else 0)
    sc_bytes = 16 * sc_a.numel()
    scale_gbs = sc_bytes / (sk["median_ms"] * 1e-3) / 1e9
    hbm_scale = {"bytes_per_call": sc_bytes, "median_ms": sk["median_ms"], "GBs": scale_gbs,
                 "frac_of_peak": scale_gbs / HBM_PEAK_GBS,
                 "machine_balance_flop_per_byte": FP64_PEAK_TFS * 1e3 / scale_gbs}
    log(f"[bench] Scale kernel over 2 x 1 GiB: {sk['median_ms']:.3f} ms, {scale_gbs:.0f} GB/s "
        f"({scale_gbs / HBM_PEAK_GBS:.2f} of peak; machine balance {FP64_PEAK_TFS * 1e3 / scale_gbs:.1f} flop/B)")
    del sc_a, sc_b

    copy_cal = None
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        cp = time_blocks(torch, lambda: b.copy_(a), 2, 1, 3)
        copy_cal = {"bytes_read": nbytes, "bytes_written": nbytes, "median_ms": cp["median_ms"],
                    "GBs_read_plus_write": 2 * nbytes / (cp["median_ms"] * 1e-3) / 1e9}
        del a, b

    if args.profile_run:
        profile_run(names, args, torch, api, synth, scale_gbs, res, copy_cal)
        return

    # ---------------------------------------------------------------- headline
    hcfg = CONFIGS[HEADLINE]
    ld = Loaded(hcfg.workload, args, torch, api, synth)
    calls = ld.calls(hcfg)

    def step():
        for _, fn in calls:
            fn()

    blocks = time_blocks(torch, step, args.steps, args.warmup, args.blocks)
    ms_per_step = blocks["median_ms"]
    value = ld.ne / (ms_per_step * 1e-3)
    log(f"[bench] headline {hcfg.name}: {blocks['blocks']} blocks of {args.steps} steps, median "
        f"{ms_per_step:.4f} ms/step (first block {blocks['first_block_ms']:.4f}, min {blocks['min_ms']:.4f}), "
        f"{value / 1e9:.2f} G elem/s fwd+VJP")
    extras = {} if args.no_extras else headline_extras(args, torch, api, ld, step)
    configs = {HEADLINE: measure_config(hcfg, ld, args, torch, api, scale_gbs, res, blocks=blocks)}
    head = configs[HEADLINE]
    ld.close()
    del ld, calls

    # ------------------------------------------------------------- the others
    loaded = {}
    order = [c for c in ("C1", "C2", "C3", "C5") if c in names]
    for i, cname in enumerate(order):
        cfg = CONFIGS[cname]
        if cfg.workload not in loaded:
            loaded[cfg.workload] = Loaded(cfg.workload, args, torch, api, synth)
        configs[cname] = measure_config(cfg, loaded[cfg.workload], args, torch, api, scale_gbs, res)
        # free a workload once no later config uses it
        if all(CONFIGS[c].workload != cfg.workload for c in order[i + 1:]):
            loaded.pop(cfg.workload).close()
            torch.cuda.empty_cache()

    wl = synth.WORKLOADS[hcfg.workload]
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
        "config": {"workload": f"{wl.name} ({HEADLINE}): {wl.n}^3-cell unit cube, 6 tets/cell, "
                               f"jitter={wl.jitter}, relabelled={wl.permute}",
                   "n_elems": head["n_elems"], "n_nodes": head["n_nodes"], "mu": wl.mu,
                   "smagorinsky_cs": wl.cs, "scatter": extras.get("scatter"),
                   "timing": f"median of {blocks['blocks']} back-to-back blocks of {args.steps} steps "
                             f"after {args.warmup} untimed steps"},
        "timing": blocks,
        "roofline": head["roofline"],
        "cpu_baseline": head.get("cpu_baseline"),
        "configs": configs,
        "hbm_scale": hbm_scale,
    }
    if copy_cal:
        result["copy_calibration"] = copy_cal
    result.update({k: v for k, v in extras.items() if k != "scatter"})
    if args.unstructured > 0:
        result["unstructured"] = unstructured_extra(args.unstructured, args, torch, api, synth)
    print(json.dumps(result), flush=True)


def unstructured_extra(n_points, args, torch, api, synth):
    """FP64 and mixed forward + velocity VJP (no eddy viscosity, mu = 1e-3) on
    the Delaunay mesh of n_points seeded uniform points: median-block rate,
    kernel durations, the mesh's layout figures and worst shape quality, and
    (with the CPU baseline) the error against the oracle."""
    t0 = time.perf_counter()
    coords, conn = synth.delaunay_mesh(n_points)
    gen_s = time.perf_counter() - t0
    ne, nn = conn.shape[0], coords.shape[0]
    d = coords[conn[:, 1:]] - coords[conn[:, :1]]
    det = np.einsum("ij,ij->i", d[:, 0], np.cross(d[:, 1], d[:, 2]))
    q_min = float(np.min(np.abs(det) / np.linalg.norm(d, axis=2).prod(axis=1)))
    del d, det
    u, p, lam = synth.unstructured_fields(coords)[:3]
    dev = torch.device("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(conn).to(dev))
    torch.cuda.synchronize()
    out = {"workload": f"delaunay of {n_points} uniform points in the unit cube", "n_elems": ne, "n_nodes": nn,
           "min_shape_quality": q_min, "mesh": mesh.info, "mesh_create_ms": (time.perf_counter() - t0) * 1e3,
           "generate_s": gen_s, "mu": 1e-3, "smagorinsky_cs": 0.0}
    log(f"[bench] unstructured: {ne} tets, {nn} nodes, generated in {gen_s:.1f} s, {mesh.info}")
    prm = api.Params(1.0, 1e-3, 0.0, synth.BODY_FORCE)
    refs = None
    if not args.no_cpu_baseline:
        import oracle

        oprm = oracle.Params(1.0, 1e-3, 0.0, synth.BODY_FORCE)
        refs = (oracle.rhs(coords, conn, u, p, oprm), oracle.vjp(coords, conn, u, lam, oprm))
    for name, dtype in (("fp64", torch.float64), ("mixed", torch.float32)):
        tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype))
        ut, pt, lt = tm(u), tm(p), tm(lam)
        rhs, grad = torch.empty_like(ut), torch.empty_like(ut)
        calls = [("fwd", lambda: api.assemble_rhs(mesh, ut, pt, prm, out=rhs)),
                 ("vjp", lambda: api.assemble_rhs_vjp(mesh, ut, lt, prm, out=grad))]

        def step():
            for _, fn in calls:
                fn()

        blocks = time_blocks(torch, step, args.steps, args.warmup, args.blocks)
        rec = {"elements_per_s": ne / (blocks["median_ms"] * 1e-3), "ms_per_step": blocks,
               "kernels": time_phases(torch, api, calls, args.steps, blocks["median_ms"])}
        if refs is not None:
            import oracle

            back = lambda t: mesh.from_mesh_order(t).double().cpu().numpy()
            rec["rel_l2_vs_oracle"] = {"rhs": oracle.rel_l2(back(rhs), refs[0]),
                                       "grad": oracle.rel_l2(back(grad), refs[1])}
        out[name] = rec
        log(f"[bench] unstructured {name}: {blocks['median_ms'] * 1e3:.1f} us/step, "
            f"{rec['elements_per_s'] / 1e9:.2f} G elem/s; "
            + ", ".join(f"{c}: {v['element_kernel_ms'] * 1e3:.1f} + {v['gather_kernel_ms'] * 1e3:.1f} us"
                        for c, v in rec["kernels"].items())
            + (f"; errors {rec['rel_l2_vs_oracle']}" if refs is not None else ""))
        del ut, pt, lt, rhs, grad
    mesh.close()
    return out


def profile_run(names, args, torch, api, synth, scale_gbs, res, copy_cal):
    """Only the listed configs, in order, without oracle: a short run for
    profiler passes (each workload's kernels dispatched a few times)."""
    args.no_cpu_baseline = True
    loaded, out = {}, {}
    for i, cname in enumerate(names):
        cfg = CONFIGS[cname]
        if cfg.workload not in loaded:
            loaded[cfg.workload] = Loaded(cfg.workload, args, torch, api, synth)
        rec = measure_config(cfg, loaded[cfg.workload], args, torch, api, scale_gbs, res)
        out[cname] = {"workload": rec["workload"], "elements_per_s": rec["elements_per_s"], "kernels": rec["kernels"]}
        if all(CONFIGS[c].workload != cfg.workload for c in names[i + 1:]):
            loaded.pop(cfg.workload).close()
            torch.cuda.empty_cache()
    print(json.dumps({"profile_run": out, "copy_calibration": copy_cal}), flush=True)


def headline_extras(args, torch, api, ld: Loaded, step):
    """On the headline mesh: the HIP-graph replay of the step, the physics
    variants and other derivative products, the autograd path, the explicit
    update, reordering and device facts."""
    u, p, lam, rhs, grad = ld.fields("fp64")
    prm, mesh, ne = ld.prm, ld.mesh, ld.ne
    dev = ld.dev
    extras = {"scatter": mesh.info["scatter"]}

    def mean_ms(fn, reps):
        """Median over five blocks of back-to-back calls (per-call mean)."""
        for _ in range(2):
            fn()
        per = max(1, reps // 5)
        out = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(per):
                fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b) / per)
        return float(np.median(out))

    # the step captured once in a HIP graph and replayed: it must reproduce
    # the eager outputs bit for bit (the gather scatter has a fixed order)
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
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(rhs, ref_rhs) and torch.equal(grad, ref_grad))
    gms = time_blocks(torch, g.replay, args.steps, 0)["median_ms"]
    extras["graph_replay"] = {"ms_per_step": gms, "elems_per_s": ne / (gms * 1e-3), "bitwise_equal_to_eager": same}
    log(f"[bench] HIP graph replay: {gms:.4f} ms/step (bitwise equal to eager: {same})")
    del g

    scratch = torch.zeros_like(u)
    acc = mesh.info["scatter"] != "patch_gather"
    variants = {}
    pr_g = torch.empty(ld.nn, dtype=torch.float64, device=dev)
    du = torch.randn_like(u)
    dpr = torch.randn_like(p)
    wl = ld.wl
    for tag, cs, model, conv in (("smagorinsky", 0.1, "smagorinsky", "advective"),
                                 ("vreman", 0.1, "vreman", "advective"),
                                 ("divergence", wl.cs, "smagorinsky", "divergence"),
                                 ("skew", wl.cs, "smagorinsky", "skew"),
                                 ("rotational", wl.cs, "smagorinsky", "rotational"),
                                 ("emac", wl.cs, "smagorinsky", "emac")):
        vp = api.Params(wl.rho, wl.mu, cs, wl.body_force, model, conv)
        tf = mean_ms(lambda: api.assemble_rhs(mesh, u, p, vp, out=scratch, accumulate=acc), args.kernel_reps)
        tv = mean_ms(lambda: api.assemble_rhs_vjp(mesh, u, lam, vp, out=scratch, accumulate=acc), args.kernel_reps)
        variants[tag] = {"eddy_model": model, "smagorinsky_cs": cs, "convective_form": conv, "fwd_ms": tf,
                         "vjp_ms": tv, "fwd_vjp_elems_per_s": ne / ((tf + tv) * 1e-3)}
    tj = mean_ms(lambda: api.assemble_rhs_jvp(mesh, u, du, dpr, prm, out=scratch, accumulate=acc), args.kernel_reps)
    tp = mean_ms(lambda: api.assemble_rhs_vjp_p(mesh, lam, prm, out=pr_g, accumulate=acc), args.kernel_reps)
    variants["jvp"] = {"ms": tj, "elems_per_s": ne / (tj * 1e-3)}
    variants["vjp_p"] = {"ms": tp, "elems_per_s": ne / (tp * 1e-3)}
    u_req = u.detach().clone().requires_grad_(True)

    def autograd_step():
        u_req.grad = None
        api.NSAssembleRHS.apply(u_req, p, mesh, prm).backward(lam)

    ta = mean_ms(autograd_step, args.kernel_reps)
    variants["autograd_fwd_bwd"] = {"ms": ta, "elems_per_s": ne / (ta * 1e-3)}
    bnd = np.any((ld.m.coords < 1e-12) | (ld.m.coords > 1 - 1e-12), axis=1)
    mask = mesh.to_mesh_order(torch.from_numpy(np.where(bnd, 7.0, 0.0)).to(dev)).to(torch.uint8)
    tu = mean_ms(lambda: api.explicit_update(mesh, u, p, prm, 1e-3, mask, out=scratch), args.kernel_reps)
    variants["explicit_update"] = {"ms": tu, "elems_per_s": ne / (tu * 1e-3),
                                   "fused": mesh.info["scatter"] == "patch_gather"}
    extras["variants"] = variants
    log("[bench] variants (fwd+vjp G elem/s): " + ", ".join(
        f"{k} {v['fwd_vjp_elems_per_s'] / 1e9:.2f}" for k, v in variants.items() if "fwd_vjp_elems_per_s" in v)
        + f"; jvp {tj * 1e3:.1f} us, vjp_p {tp * 1e3:.1f} us, explicit update {tu * 1e3:.1f} us, "
        f"autograd forward + backward {ta * 1e3:.1f} us")

    # the immediate atomic scatter of the paper's final kernel on its own:
    # device-scope atomic adds into an (Nn, 3) vector, 4 Ne index entries x 3
    # components (the atomics of one atomic-scatter assembly call), FP64 and
    # FP32, for three index patterns
    conn_m, _ = mesh.connectivity()
    n_idx = 4 * ne
    k = torch.arange(n_idx, device=dev, dtype=torch.int64)
    patterns = {"mesh_connectivity": conn_m.reshape(-1).contiguous(),
                "contiguous": (k % ld.nn).to(torch.int32),
                "strided_4099": ((k * 4099) % ld.nn).to(torch.int32)}
    del k, conn_m
    atom = {"atomics_per_call": 3 * n_idx, "rows": ld.nn}
    for dt, tag in ((torch.float64, "fp64"), (torch.float32, "fp32")):
        acc_buf = torch.zeros((ld.nn, 3), dtype=dt, device=dev)
        for name, idx in patterns.items():
            t = mean_ms(lambda: api.scatter_add(idx, acc_buf), 10)
            atom[f"{tag}_{name}"] = {"ms": t, "atomics_per_s": 3 * n_idx / (t * 1e-3),
                                     "ns_per_element_12_atomics": t * 1e6 / ne}
        del acc_buf
    del patterns
    extras["atomic_scatter"] = atom
    log("[bench] atomic scatter (G atomics/s): " + ", ".join(
        f"{k_}: {v['atomics_per_s'] / 1e9:.1f}" for k_, v in atom.items() if isinstance(v, dict)))

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    u_user = torch.from_numpy(np.ascontiguousarray(ld.u)).to(dev)
    mesh.to_mesh_order(u_user)
    start.record()
    mesh.to_mesh_order(u_user)
    stop.record()
    torch.cuda.synchronize()
    extras["setup"] = {"mesh_create_ms": ld.create_ms, "to_mesh_order_ms_per_vector_field": start.elapsed_time(stop),
                       "device": torch.cuda.get_device_name(dev), "hip": getattr(torch.version, "hip", None)}
    return extras


if __name__ == "__main__":
    main()
