"""Benchmark of the emRKC hot path on one MI355X.

One bench step is one whole simulation of the large slab workload (the
largest configuration that fits one GPU: 601 x 601 x 101 Q1 nodes =
36,481,301 nodes, CRN surrogate with 21 variables, planar stimulus on the
x = 0 face, dt = 0.05 ms, T = 20 ms): resting-state initialisation,
spectral-radius estimation by power iteration, and 400 emRKC steps (outer
RKC stages with the fused ionic/Rush-Larsen head kernel and the inner
diffusion stages), replayed from HIP graphs.  Throughput is node-steps per
second of the whole job.  The same line carries the dominant kernel's
roofline (timed with HIP events in a separate pass of eagerly launched
kernels), the measured copy and 3-read/1-write stream bandwidths of the
device, the mixed FP32 form with its error in V, and the FP64 oracle timed
on the host cores.  On the slab the solution depends on x alone, so the
oracle's run on the 601 x 2 x 2 reduction of the same grid gives the exact
reference V at T for every node; the error of both forms against it is
reported.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X vector FP64, published
METRIC = "node-steps/s emRKC on 1 GPU, % HBM roofline; FP32 vs FP64 at stated V error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_node(kind, nz, wz, m, mat=0):
    """Algorithmic HBM bytes per node of one launch (s = 1): V and u values
    are doubles, z has width wz, S_V has width sv (4 in the mixed form), and
    every diffusion product on an unstructured mesh adds the ELL row `mat`
    (column indices and weights; 0 on grids, whose stencil is implicit).
    head : V (8), z read and written (2 nz wz), S_V (sv) and u_1 (8) written;
           with m == 1 it writes V_{n+1} (8) instead of S_V and u_1
    fused: last inner stage of the previous step -- u_{m-1} (8), u_{m-2} (8,
           only when m >= 3: for m = 2 it is V), V (8), S_V (sv) -- plus the
           head without its V read, plus V^n written (8)
    inner: u_{k-1}, u_{k-2}, S_V, u_k
    tail : u_{m-1}, u_{m-2} (m >= 3), V, S_V, V written"""
    sv = 4 if wz == 4 else 8
    if kind == "head":
        return 8 + 2 * nz * wz + (8 if m == 1 else sv + 8) + mat
    # the split stage (m >= 2, 3-D grids): the pointwise head reads V and z,
    # writes z and S_V; the two-stage inner kernel reads V (u_0) and S_V and
    # writes V_j (m == 2) or u_1 and u_2 (m >= 3)
    if kind == "head_pw":
        return 8 + 2 * nz * wz + sv
    if kind == "inner12":
        return 8 + sv + (8 if m == 2 else 16)
    # u_1 as an inner-kernel launch (head shape 8): reads u_0 = V and S_V, writes u_1
    if kind == "inner1":
        return 8 + sv + 8
    if kind == "fused":
        return 8 + (8 if m >= 3 else 0) + 8 + sv + 2 * nz * wz + sv + 8 + 8 + 2 * mat
    # 2-D grids, all inner stages of a stage in one launch: u_1, V and S_V
    # read (with halos staged in LDS), V_j written; u_2 .. u_{m-1} never
    # leave LDS.  One kernel per step adds the next step's head without its
    # V read: z read and written, S_V and u_1 written
    if kind == "inner_all":
        return 8 + 8 + sv + 8
    if kind == "step2d":
        return 8 + 8 + sv + 8 + 2 * nz * wz + sv + 8
    if kind == "inner":
        return 8 + 8 + sv + 8 + mat
    if kind == "tail":
        return 8 + (8 if m >= 3 else 0) + 8 + sv + 8 + mat
    # mRKC (FP64): the head reads V and z, writes z except the stiffest gate,
    # S_V, u_1 and w_1 (gate 0); the last inner stage (m = 2) reads u_1, V,
    # S_V, w_1 and gate 0 of z, writes V and gate 0
    if kind == "mrkc_head":
        return 8 + 8 * nz + 8 * (nz - 1) + 8 + 8 + 8 + mat
    if kind == "mrkc_tail":
        return 8 + 8 + 8 + 8 + 8 + 8 + 8 + mat
    # IMEX-RL (FP64 solve); dsum = 8 on unstructured meshes (the row sums of
    # the preconditioner), 0 on grids (one value)
    #   pointwise: V read, z read and written, right-hand side written
    #   cg_init  : x, b, ML (+ D) read, r, z written
    #   cg_apply : z, previous p, ML read, p and q written (the new
    #              direction and the operator product in one kernel)
    #   cg_update: x, r read and written, p, q, ML (+ D) read, z written
    dsum = 8 if mat else 0
    if kind == "cg_pointwise":
        return 8 + 2 * nz * wz + 8
    if kind == "cg_init":
        return 8 + 8 + 8 + dsum + 16 + mat
    if kind == "cg_apply":
        return 8 + 8 + 8 + 16 + mat
    if kind == "cg_update":
        return 16 + 16 + 8 + 8 + 8 + dsum + 8
    raise ValueError(kind)


class Job:
    def __init__(self, cfg, precision, stream, flags=0, tet=None, batch=None, method="emrkc"):
        from paper_2401_01745_amd import emrkc as E
        self.E = E
        self.cfg = cfg
        # IMEX-RL is a separate entry point on a plain (emRKC) context
        cmethod = "emrkc" if method == "imexrl" else method
        if batch is not None:
            self.sim = E.simulation_from_batch(batch, precision=precision, flags=flags)
        elif tet is not None:
            self.sim = E.simulation_from_tet_config(cfg, tet[0], tet[1], precision=precision, flags=flags,
                                                    method=cmethod)
        else:
            self.sim = E.simulation_from_config(cfg, precision=precision, flags=flags, method=cmethod)
        E.emrkc_set_stream(self.sim.ctx, stream.cuda_stream)
        self.nsim = int(round(cfg["T"] / cfg["dt"]))
        self.method = method

    def tune(self, variants=None):
        """Kernel shapes: given, or chosen by the library's autotuner on the
        resting state (outside the timed region, like compilation)."""
        E, s = self.E, self.sim
        if self.method == "imexrl":
            return None
        if variants is not None:
            E.emrkc_set_variants(s.ctx, variants)
            return tuple(variants)
        E.emrkc_init_state(s.ctx, s.state)
        E.emrkc_estimate_rho(s.ctx, s.state)
        return E.emrkc_autotune(s.ctx, s.state, self.cfg["dt"], reps=10)

    def run(self):
        E, s = self.E, self.sim
        s.state.t0 = 0.0
        s.state.step = 0
        E.emrkc_init_state(s.ctx, s.state)
        if self.method == "imexrl":
            E.emrkc_imexrl_step(s.ctx, s.state, self.cfg["dt"], self.nsim)
            return E.emrkc_imexrl_iterations(s.ctx)
        rF, rS, itF, itS, _ = E.emrkc_estimate_rho(s.ctx, s.state)
        E.emrkc_step(s.ctx, s.state, self.cfg["dt"], self.nsim)
        return rF, rS, itF, itS


def time_jobs(job, warmup, steps, torch):
    for _ in range(warmup):
        job.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = job.run()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, info


# Largest grid the CPU leg assembles whole (nodes).  Beyond it the oracle is
# timed on a sub-slab of the first planes of the same grid: assembling the
# 36.5M-node slab takes the oracle about 2.5 minutes and 55 GB, and one of
# its steps about half a minute.
CPU_MAX_NODES = 2_000_000


def cpu_sample_config(cfg):
    """The workload the CPU leg times: cfg itself, or for a 3-D grid above
    CPU_MAX_NODES its first k z-planes (same spacing, conductivity, model
    and stimulus rule), with k the largest that stays within the bound."""
    if cfg.get("kind") != "grid" or int(np.prod(cfg["n"])) <= CPU_MAX_NODES or cfg["dim"] != 3:
        return cfg, None
    n0, n1, n2 = cfg["n"]
    k = max(2, min(n2, CPU_MAX_NODES // (n0 * n1)))
    return dict(cfg, n=(n0, n1, k)), k


def cpu_baseline(cfg, seconds, tet=None, method="emrkc"):
    """The FP64 oracle on the same workload, timed for a bounded number of
    emRKC (or mRKC) steps (assembly and radii excluded), on the full mesh or
    on the sub-slab of cpu_sample_config.  For the ensemble the sample is
    its first instance."""
    from oracle.emrkc import emrkc_step, stage_counts
    from oracle.monodomain import build_grid_problem, build_tet_problem
    from oracle.mrkc import MrkcSplit, mrkc_step
    from oracle.powiter import compute_rho, random_unit_interval
    if tet is not None:
        prob = build_tet_problem(cfg, *tet)
    else:
        cfg, _ = cpu_sample_config(cfg)
        prob = build_grid_problem(cfg, stim_mask=cfg.get("mask"))
    y = prob.uniform_state()
    v0 = random_unit_interval(y.size, 0)
    split = MrkcSplit(prob) if method == "mrkc" else prob
    _, rF, _, _ = compute_rho(0.0, y, split.f_F, v0.copy())
    _, rS, _, _ = compute_rho(0.0, y, split.f_S, v0.copy())
    rF, rS = 1.05 * rF, 1.05 * rS
    n = 0
    t0 = time.perf_counter()
    while True:
        if method == "mrkc":
            y = mrkc_step(n * cfg["dt"], y, cfg["dt"], split.f_F, split.f_S, rF, rS)
        else:
            y = emrkc_step(n * cfg["dt"], y, cfg["dt"], prob, rF, rS)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    return prob.N * n / el, n, el, stage_counts(cfg["dt"], rF, rS), prob.N


def planar_reduction(cfg):
    """For a 3-D grid whose stimulus is a whole x-face band (uniform in y
    and z) and whose initial state is uniform, the solution depends on x
    alone: the zero-flux Q1 operator maps a field constant in y and z to
    the operator of the n0 x 2 x 2 grid of the same spacing (the y and z
    difference terms vanish, the mirrored mass weights sum to one).  Returns
    that reduced workload, or None when the reduction does not apply."""
    st = cfg.get("stim", {})
    if cfg.get("kind") != "grid" or cfg.get("dim") != 3 or st.get("kind") != "face" or st.get("axis") != 0:
        return None
    return dict(cfg, n=(cfg["n"][0], 2, 2), name=cfg["name"] + "_x_reduction")


def oracle_reference_V(cfg, nsteps, rho_F, rho_S):
    """V at T from the FP64 oracle on the reduction of planar_reduction
    (an x-profile of n0 values), run with the given radii (the method uses
    them only through its stage counts (s, m)), or None."""
    red = planar_reduction(cfg)
    if red is None:
        return None
    from oracle.emrkc import emrkc_run
    from oracle.monodomain import build_grid_problem
    prob = build_grid_problem(red)
    y = emrkc_run(prob, prob.uniform_state(), 0.0, cfg["dt"], nsteps, rho_F, rho_S)
    return y[:prob.N].reshape(2, 2, cfg["n"][0])[0, 0].copy()


def errors_vs_profile(V, ref, n, torch):
    """(relative L2, relative max) of the device vector V on an n0 x n1 x n2
    grid against the x-profile ref broadcast over y and z."""
    r = torch.from_numpy(ref).to(V.device)
    d = V.view(n[2], n[1], n[0]) - r.view(1, 1, -1)
    ref_l2 = float(np.linalg.norm(ref)) * float(np.sqrt(n[1] * n[2]))
    return float(torch.linalg.vector_norm(d).item()) / ref_l2, float(d.abs().max().item()) / float(np.abs(ref).max())


def stream_bandwidth(torch, stream, mib=1024, reps=5):
    """GB/s of a 3-read/1-write stream over FP64 vectors of `mib` MiB each
    (d = a + b c, torch's addcmul), best of `reps`: the traffic pattern of
    the inner stages, as a practical ceiling next to the plain copy."""
    n = mib << 17
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    d = torch.empty_like(a)
    torch.addcmul(a, b, c, out=d)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        torch.addcmul(a, b, c, out=d)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    assert float(d[n // 2].item()) == 2.0
    del a, b, c, d
    torch.cuda.empty_cache()
    return 4.0 * (mib << 20) / (best * 1e-3) / 1e9


def copy_bandwidth(torch, stream, mib=1024, reps=5):
    """GB/s (read + write bytes) of torch's device-to-device copy of `mib` MiB."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dst.copy_(src)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5_3d_crn_large")
    ap.add_argument("--kernel-steps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--method", default="emrkc", choices=["emrkc", "mrkc", "imexrl"],
                    help="mrkc: the mRKC method (stiffest gate in the fast term), FP64, flat kernels; "
                         "imexrl: the IMEX-RL method (implicit diffusion by preconditioned CG), FP64")
    ap.add_argument("--variants", default=None,
                    help="kernel shapes 'head,head_planes,inner,inner_planes,fused' instead of autotuning")
    ap.add_argument("--z-layout", default="auto", choices=["auto", "blocks", "planes"],
                    help="ionic state layout while stepping: the library's choice (blocks of 256 nodes for z "
                         "arrays of 256 MiB and more), or forced; counted traffic is reported for auto only")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy a buffer of this size once (calibrates rocprof FETCH/WRITE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the emRKC hot path here is a single-GPU build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_01745_amd import emrkc as E
    from workloads.configs import get_config
    E.lib()
    torch.cuda.set_device(0)
    tet = None
    batch = None
    if args.config.startswith("c4"):
        from workloads.ensemble import ensemble
        batch = ensemble()
        cfg = dict(batch[0], name="c4_ensemble64", T=batch[0]["T"])
        N = int(sum(np.prod(c["n"]) for c in batch))
    elif args.config.startswith("c3"):
        from workloads.tetmesh import build_shell, shell_config
        cfg = shell_config()
        tet = build_shell(cfg)
        N = tet[0]["coords"].shape[0]
    else:
        cfg = get_config(args.config)
        N = int(np.prod(cfg["n"]))
    stream = torch.cuda.Stream()
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: calibration copy of %d MiB done" % args.calib_copy_mib)
        del src, dst
    if args.method == "imexrl":
        if batch is not None:
            print("bench.py: IMEX-RL runs single contexts only (not the ensemble)", file=sys.stderr)
            sys.exit(2)
        with torch.cuda.stream(stream):
            out = bench_imexrl(args, cfg, N, tet, stream, E, torch)
        print(json.dumps(out), flush=True)
        return
    with torch.cuda.stream(stream):
        log("bench: %s, N=%d, building FP64 context" % (cfg["name"], N))
        flags = {"auto": 0, "blocks": E.EMRKC_Z_BLOCKS, "planes": E.EMRKC_Z_PLANES}[args.z_layout]
        job = Job(cfg, "fp64", stream, flags, tet, batch, method=args.method)
        forced = tuple(int(x) for x in args.variants.split(",")) if args.variants else None
        variants = job.tune(forced)
        log("bench: fp64 kernel shapes %s" % (variants,))
        elapsed, (rF, rS, itF, itS) = time_jobs(job, args.warmup, args.steps, torch)
        z_blocks = bool(E.emrkc_last_stats(job.sim.ctx).z_blocks)  # the layout the timed steps used
        s, m, eta = E.emrkc_stages(job.sim.ctx, cfg["dt"])
        value = N * job.nsim * args.steps / elapsed
        log("bench: fp64 %.3f ms per simulation (%d steps), %.4g node-steps/s, s=%d m=%d" %
            (1e3 * elapsed / args.steps, job.nsim, value, s, m))
        V64 = job.sim.V.clone()
        radii64 = E.emrkc_get_rho(job.sim.ctx)

        # per-launch kernel durations: HIP events around every kernel on the
        # job's stream, over kernel-steps further steps of the same
        # simulation (eager launches of the kernels the timed graphs replay)
        prof = E.emrkc_profile_step(job.sim.ctx, job.sim.state, cfg["dt"], args.kernel_steps)
        nz = job.sim.nv - 1
        log("bench: kernel means (ms, launches): %s" % prof)
        dom = "fused" if prof["fused"][1] > prof["head"][1] else "head"
        dom_ms = prof[dom][0]
        # the split stage: pointwise head + two-stage inner kernel (shape 7)
        split = batch is None and tet is None and args.method == "emrkc" and variants[0] in (7, 8) and m >= 2
        # 2-D grids: all inner stages in one launch (inner shapes 2, 3), or
        # one kernel per step (shape 4, whose launches are the fused class)
        planar2d = (batch is None and tet is None and args.method == "emrkc" and cfg.get("dim") == 2
                    and variants[2] in (2, 3, 4) and m >= 2)
        step2d = planar2d and variants[2] == 4
        width = E.lib().emrkc_ell_width(job.sim.ctx) if tet is not None else 0
        mat = width * (4 + 8)
        if batch is not None:
            off, ms, _, _ = E.emrkc_batch_info(job.sim.ctx, cfg["dt"])
            sizes = np.diff(off)
            db = int(sum(n * bytes_per_node("head", nz, 8, mk) for n, mk in zip(sizes, ms)))
        elif args.method == "mrkc":
            db = bytes_per_node("mrkc_head", nz, 8, m, mat) * N
        elif split:
            db = bytes_per_node("head_pw", nz, 8, m) * N
        elif step2d and dom == "fused":
            db = bytes_per_node("step2d", nz, 8, m) * N
        else:
            db = bytes_per_node(dom, nz, 8, m, mat) * N
        dom_gbs = db / (dom_ms * 1e-3) / 1e9
        # HBM bytes per launch from the committed rocprof counters, when they
        # were taken on these library sources for the kernel shape chosen here
        prof_path = os.path.join(ROOT, "profiles", "traffic_k_%s%s_%s_fp64.json"
                                 % ("mrkc_" if args.method == "mrkc" else "", dom, cfg["name"]))
        traffic = None
        valu = None
        tr_ok = None  # the counters file, when taken on these sources
        if args.method in ("emrkc", "mrkc") and args.z_layout == "auto" and os.path.exists(prof_path):
            tr = json.load(open(prof_path))
            ent = tr.get("by_shape", {}).get("%d,%d,%d" % (variants[0], variants[1], variants[4]))
            if tr.get("kernel_source_hash") == kernel_hash() and ent is not None:
                tr_ok = tr
                traffic = ent.get("bytes_per_launch")
                if "valu_busy" in ent:
                    # the FP64 vector ALU side of the same kernel (rocprof
                    # SQ_INSTS_VALU over its profiled duration; one wave64
                    # instruction per 4 cycles on 1024 SIMDs at 2.4 GHz)
                    valu = {"instr_per_wave": ent["valu_instr_per_wave"], "busy_frac": ent["valu_busy"],
                            "peak": "78.6 TFLOP/s FP64 vector", "source": tr.get("source")}
        head_kernel = ("k_mrkc_head" if args.method == "mrkc" else
                       ("k_head_batch_flat" if variants[1] else "k_head_batch<tile shape %d>" % variants[0])
                       if batch is not None else
                       "k_head" if tet is not None else
                       {0: "k_head_tiled", 1: "k_head_march", 2: "k_head_march_lds", 3: "k_head_tiled_occ<6 waves/SIMD>",
                        4: "k_head_tiled_occ<8 waves/SIMD>", 5: "k_head (flat)",
                        6: "k_head_occ (flat, 7 waves per SIMD)", 7: "k_head_pw (pointwise)",
                        8: "k_head_pw (pointwise)"}[variants[0]])
        names = {"fused": "k_step2d (all inner stages and the outer V update of step n-1 + exponential Euler, "
                          "ionic model, outer z recurrence and first inner stage of step n)" if step2d else
                          "k_fused (last inner stage of step n-1 + exponential Euler, ionic model, outer z "
                          "recurrence and first inner stage of step n)",
                 "head": ("%s (exponential Euler, ionic model, outer z recurrence, S_V)" % head_kernel if split else
                          "%s (exponential Euler, ionic model, outer z recurrence, first inner stage)" % head_kernel)
                 if args.method == "emrkc" else
                 "%s (ionic model and gate rates, outer z recurrence, first inner stage of V and the stiffest "
                 "gate)" % head_kernel}
        # the inner kernel in this pass is the last inner stage (stencil +
        # Chebyshev recurrence + outer V update) when m == 2
        if batch is not None:
            ib = int(sum(n * bytes_per_node("tail", nz, 8, 2) for n, mk in zip(sizes, ms) if mk == 2))
        elif split and variants[0] == 7:
            ib = bytes_per_node("inner12", nz, 8, m) * N if m == 2 else None
        elif split:  # u_1 launch and the last inner stage, mean bytes per launch
            ib = (bytes_per_node("inner1", nz, 8, m) + bytes_per_node("tail", nz, 8, m)) * N // 2 if m == 2 else None
        elif planar2d:  # all inner stages in one launch (s == 1); with shape 4 only the chunk's last step
            ib = bytes_per_node("inner_all", nz, 8, m) * N if s == 1 else None
        elif args.method == "mrkc":
            ib = bytes_per_node("mrkc_tail", nz, 8, m, mat) * N if m == 2 else None
        else:
            ib = bytes_per_node("tail" if m == 2 else "inner", nz, 8, m, mat) * N
        inner_gbs = ib / (prof["inner"][0] * 1e-3) / 1e9 if prof["inner"][1] and ib else None
        roof = {"kernel": names[dom], "bound": "hbm", "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": db, "launch_ms": round(dom_ms, 5), "valu": valu,
                "kernels_ms": {k: round(v[0], 5) for k, v in prof.items()},
                "launches": {k: v[1] for k, v in prof.items()},
                "inner_stencil_kernel": {"kernel": "k_inner12_march (first two inner stages and the outer V update)"
                                         if split and variants[0] == 7 else
                                         "k_inner_all2d (all %d inner stages and the outer V update, %dx%d tiles)"
                                         % (m - 1, 16 if variants[2] == 2 else 8, 16 if variants[2] == 2 else 8)
                                         if planar2d else
                                         "first inner stage and last inner stage with the outer V update (mean)"
                                         if split else "last inner stage and the outer V update",
                                         "achieved_GBs": round(inner_gbs, 1) if inner_gbs else None,
                                         "frac": round(inner_gbs / HBM_PEAK_GBS, 4) if inner_gbs else None,
                                         "bytes_per_launch": ib,
                                         "traffic": counted(tr_ok, "inner", variants)}}

        mixed = None
        if not args.no_mixed and args.method == "emrkc":
            log("bench: mixed FP32 form")
            jm = Job(cfg, "mixed", stream, flags, tet, batch)
            variants_m = jm.tune(forced)
            log("bench: mixed kernel shapes %s" % (variants_m,))
            el_m, _ = time_jobs(jm, 1, max(1, args.steps // 2), torch)
            value_m = N * jm.nsim * max(1, args.steps // 2) / el_m
            Vm = jm.sim.V.clone()
            radiim = E.emrkc_get_rho(jm.sim.ctx)
            sm_m = E.emrkc_stages(jm.sim.ctx, cfg["dt"])[:2]
            d = Vm - V64
            # the mixed form's head kernel: its own launch time and algorithmic
            # bandwidth (z and S_V in float; ELL weights in float on tets)
            pm = E.emrkc_profile_step(jm.sim.ctx, jm.sim.state, cfg["dt"], args.kernel_steps)
            mat_m = width * (4 + 4)
            if batch is not None:
                off_m, ms_m, _, _ = E.emrkc_batch_info(jm.sim.ctx, cfg["dt"])
                dbm = int(sum(n * bytes_per_node("head", nz, 4, mk) for n, mk in zip(np.diff(off_m), ms_m)))
            else:
                mm = E.emrkc_stages(jm.sim.ctx, cfg["dt"])[1]
                split_m = tet is None and variants_m[0] in (7, 8) and mm >= 2
                dbm = bytes_per_node("head_pw" if split_m else "head", nz, 4, mm, mat_m) * N
            head_m = {"launch_ms": round(pm["head"][0], 5), "bytes_per_launch": dbm,
                      "achieved_GBs": round(dbm / (pm["head"][0] * 1e-3) / 1e9, 1),
                      "frac": round(dbm / (pm["head"][0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)} if pm["head"][1] else None
            inner_m = None
            if batch is None and pm["inner"][1]:
                mm = E.emrkc_stages(jm.sim.ctx, cfg["dt"])[1]
                ibm = (bytes_per_node("inner12", nz, 4, mm) if (tet is None and variants_m[0] == 7 and mm == 2) else
                       (bytes_per_node("inner1", nz, 4, mm) + bytes_per_node("tail", nz, 4, mm)) // 2
                       if (tet is None and variants_m[0] == 8 and mm == 2) else
                       bytes_per_node("tail", nz, 4, mm, mat_m) if mm == 2 else None)
                if ibm:
                    inner_m = {"launch_ms": round(pm["inner"][0], 5), "bytes_per_launch": ibm * N,
                               "achieved_GBs": round(ibm * N / (pm["inner"][0] * 1e-3) / 1e9, 1)}
            if head_m is not None:
                head_m["traffic"] = counted(tr_ok, "mixed", variants_m, "head")
            if inner_m is not None:
                inner_m["traffic"] = counted(tr_ok, "mixed", variants_m, "inner")
            mixed = {"value": value_m, "speedup_vs_fp64": round(value_m / value, 3), "kernel_shapes": variants_m,
                     "head_kernel": head_m, "inner_kernel": inner_m,
                     "s_m": list(sm_m),
                     "V_rel_l2_vs_fp64": float(torch.linalg.vector_norm(d).item() /
                                               torch.linalg.vector_norm(V64).item()),
                     "V_rel_max_vs_fp64": float(d.abs().max().item() / V64.abs().max().item()),
                     "V_rel_l2_vs_oracle": None, "V_rel_max_vs_oracle": None,
                     "reference": "GPU FP64 path at T (matches the FP64 oracle to 1e-10 in the parity tests)"}
            del d
            log("bench: mixed %.4g node-steps/s, V rel L2 %.3e" % (value_m, mixed["V_rel_l2_vs_fp64"]))
            jm.sim.close()
        job.sim.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

    # the practical bandwidth ceiling on this GPU: a plain device-to-device
    # copy of 1 GiB (the HIP runtime's copy kernel), best of 5, timed on the
    # same stream outside the timed region
    with torch.cuda.stream(stream):
        copy_gbs = copy_bandwidth(torch, stream)
        stream_gbs = stream_bandwidth(torch, stream)
    roof["copy_GBs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    roof["stream3r1w_GBs"] = round(stream_gbs, 1)
    roof["frac_of_stream"] = round(roof["achieved"] / stream_gbs, 4)
    log("bench: device copy %.1f GB/s, 3-read/1-write stream %.1f GB/s; dominant kernel at %.1f%% / %.1f%% of them"
        % (copy_gbs, stream_gbs, 100 * roof["frac_of_copy"], 100 * roof["frac_of_stream"]))

    mname = "mRKC" if args.method == "mrkc" else "emRKC"
    cpu = None
    fp64_err = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        v, n, el, sm, Ns = cpu_baseline(cfg, args.cpu_seconds, tet, args.method)
        sub = cpu_sample_config(cfg)[1] if (tet is None and batch is None) else None
        what = (("the full %d-node mesh" % Ns) if Ns == N else
                ("the first %d z-planes of the grid (%s, %d nodes)"
                 % (sub, "x".join(map(str, cpu_sample_config(cfg)[0]["n"])), Ns)) if sub else
                ("instance 0 (%d nodes) of the ensemble" % Ns))
        cpu = {"value": v, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
               "sample": "%d %s steps of %s in %.1f s (numpy/scipy, single thread; host has %d logical CPUs)"
                         % (n, mname, what, el, os.cpu_count())}
        # the oracle's V at T on the x-reduction of a planar-wave grid: the
        # error of both forms in every node at the full length of the run
        if args.method == "emrkc" and planar_reduction(cfg) is not None:
            log("bench: FP64 oracle on the %s reduction, %d steps" % ("x".join(map(str, planar_reduction(cfg)["n"])),
                                                                     job.nsim))
            ref = oracle_reference_V(cfg, job.nsim, *radii64)
            e2, emax = errors_vs_profile(V64, ref, cfg["n"], torch)
            fp64_err = {"V_rel_l2_vs_oracle": e2, "V_rel_max_vs_oracle": emax, "s_m": [s, m],
                        "reference": "FP64 oracle on the %s grid (the planar wave depends on x alone), %d steps"
                                     % ("x".join(map(str, planar_reduction(cfg)["n"])), job.nsim)}
            log("bench: fp64 V vs oracle: rel L2 %.3e, rel max %.3e" % (e2, emax))
            if mixed is not None:
                if tuple(mixed["s_m"]) != (s, m):
                    ref = oracle_reference_V(cfg, job.nsim, *radiim)
                e2, emax = errors_vs_profile(Vm, ref, cfg["n"], torch)
                mixed.update(V_rel_l2_vs_oracle=e2, V_rel_max_vs_oracle=emax, reference=fp64_err["reference"])
                log("bench: mixed V vs oracle: rel L2 %.3e, rel max %.3e" % (e2, emax))

    out = {"metric": METRIC.replace("emRKC", mname), "value": value, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "%s: %s (%d nodes), %s, chi=%g/mm, Cm=%g uF/mm^2, sigma=%s, dt=%g ms, "
                                  "T=%g ms; one bench step = init + power iteration + %d %s steps"
                                  % (cfg["name"], ("P1 tetrahedral shell %s" % "x".join(map(str, cfg["dims"])))
                                     if tet is not None else
                                     ("ensemble of %d 2-D/3-D Q1 slabs, one batched context" % len(batch))
                                     if batch is not None else ("Q1 grid %s" % "x".join(map(str, cfg["n"]))),
                                     N, cfg["model"], cfg["chi"], cfg["Cm"], list(cfg["sigma"]), cfg["dt"], cfg["T"],
                                     job.nsim, mname),
                      "method": args.method, "kernel_shapes": variants, "s": s, "m": m, "eta": eta, "rho_F": rF, "rho_S": rS, "powiter_iters": [itF, itS],
                      "z_layout": "blocks of 256 nodes" if z_blocks else "component planes"},
           "roofline": roof, "fp64_error": fp64_err, "mixed": mixed, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def cpu_baseline_imexrl(cfg, seconds, tet=None):
    """The FP64 oracle's IMEX-RL step for a bounded number of steps on the
    full mesh, its implicit line solved by scipy's Jacobi-preconditioned
    conjugate gradients on the symmetric form (a sparse LU of the 3-D
    operator takes minutes to factorise at these sizes)."""
    from oracle.exexrl import imexrl_cg_solver, imexrl_step
    from oracle.monodomain import build_grid_problem, build_tet_problem
    prob = build_tet_problem(cfg, *tet) if tet is not None else build_grid_problem(cfg, stim_mask=cfg.get("mask"))
    solve = imexrl_cg_solver(cfg["dt"], prob)
    y = prob.uniform_state()
    n = 0
    t0 = time.perf_counter()
    while True:
        y = imexrl_step(n * cfg["dt"], y, cfg["dt"], prob, solve)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    return prob.N * n / el, n, el, prob.N


IMEXRL_KERNEL_NAMES = {"pointwise": "k_imexrl_pre", "cg_init": "k_cg_init",
                       "cg_apply": "k_cg_dir_apply (new direction and operator product)",
                       "cg_update": "k_cg_update"}


def bench_imexrl(args, cfg, N, tet, stream, E, torch):
    """IMEX-RL on the same workload: one bench step is one whole simulation
    (resting state, T/dt steps, each a pointwise Rush-Larsen kernel and a
    conjugate-gradient solve of the implicit diffusion line)."""
    log("bench: %s, N=%d, IMEX-RL (FP64)" % (cfg["name"], N))
    job = Job(cfg, "fp64", stream, 0, tet, None, method="imexrl")
    elapsed, iters = time_jobs(job, args.warmup, args.steps, torch)
    value = N * job.nsim * args.steps / elapsed
    log("bench: imexrl %.3f ms per simulation (%d steps, %d CG iterations), %.4g node-steps/s" %
        (1e3 * elapsed / args.steps, job.nsim, iters, value))
    ksteps = max(1, min(args.kernel_steps // 4, job.nsim))
    prof = E.emrkc_profile_imexrl(job.sim.ctx, job.sim.state, cfg["dt"], ksteps)
    log("bench: kernel means (ms, launches): %s" % prof)
    nz = job.sim.nv - 1
    width = E.lib().emrkc_ell_width(job.sim.ctx) if tet is not None else 0
    mat = width * (4 + 8)

    def kbytes(k):
        return bytes_per_node("cg_" + k.replace("cg_", ""), nz, 8, 0, mat) * N

    total = {k: v[0] * v[1] for k, v in prof.items()}
    dom = max(total, key=total.get)
    dom_gbs = kbytes(dom) / (prof[dom][0] * 1e-3) / 1e9
    roof = {"kernel": IMEXRL_KERNEL_NAMES[dom], "bound": "hbm", "achieved": round(dom_gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": kbytes(dom), "launch_ms": round(prof[dom][0], 5),
            "kernels_ms": {k: round(v[0], 5) for k, v in prof.items()},
            "launches": {k: v[1] for k, v in prof.items()},
            "kernels_GBs": {k: round(kbytes(k) / (v[0] * 1e-3) / 1e9, 1) for k, v in prof.items() if v[1]}}
    job.sim.close()
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (IMEX-RL)")
        v, n, el, Ns = cpu_baseline_imexrl(cfg, args.cpu_seconds, tet)
        cpu = {"value": v, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
               "sample": "%d IMEX-RL steps of the full %d-node mesh in %.1f s (numpy/scipy, CG solves to "
                         "1e-13, single thread; host has %d logical CPUs)" % (n, Ns, el, os.cpu_count())}
    mesh = (("P1 tetrahedral shell %s" % "x".join(map(str, cfg["dims"]))) if tet is not None
            else ("Q1 grid %s" % "x".join(map(str, cfg["n"]))))
    return {"metric": METRIC.replace("emRKC", "IMEX-RL"), "value": value, "unit": "node-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "%s: %s (%d nodes), %s, dt=%g ms, T=%g ms; one bench step = init + %d IMEX-RL "
                                   "steps" % (cfg["name"], mesh, N, cfg["model"], cfg["dt"], cfg["T"], job.nsim),
                       "method": "imexrl", "cg_iterations_per_simulation": iters, "cg_tolerance": 1e-13},
            "roofline": roof, "cpu_baseline": cpu}


def counted(tr, part, variants, sub=None):
    """HBM bytes per launch from the committed counters (None when they were
    not taken on these library sources or for these kernel shapes)."""
    if tr is None:
        return None
    ent = tr.get(part, {}).get("%d,%d,%d" % (variants[0], variants[1], variants[4]))
    if ent is not None and sub is not None:
        ent = ent.get(sub)
    return ent.get("bytes_per_launch") if ent else None


def kernel_hash():
    """Hash of the library's sources: the kernels and the host code, which
    chooses their launch shapes and the data layout they read (z in blocks
    or in component planes)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("emrkc_kernels.hip", "emrkc_device.h", "emrkc_internal.h", "emrkc_host.hip"):
        h.update(open(os.path.join(ROOT, "paper_2401_01745_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
