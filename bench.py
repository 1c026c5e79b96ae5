#!/usr/bin/env python3
"""Throughput of C-A CUR low-rank approximation on one MI355X.

Workload: one 20000 x 20000 FP32 matrix A = X Y / ||X Y||_F + N(0, 1e-6^2)
(X, Y Gaussian, rank 50), abridged SRHT start (depth 3, 100 sampled columns),
rank 50, 4 C-A sweeps, FP64 panels and nucleus.  One step = one whole LRA
(sketch, QRP seed, sweeps, nucleus) with A already resident in HBM.

Prints one JSON line.  The roofline block is for the persistent C-A kernel
(the only kernel of a step besides a one-workgroup counter reset); its bytes
are the algorithmic reads of the LRA divided by its measured duration.  The
cpu_baseline block times the FP64 CPU oracle on the same matrix.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M = N = 20000
RANK = 50
SWEEPS = 4
DEPTH = 3
SAMPLES = 100
SEED = 2011
METRIC = "CUR LRAs/sec + HBM GB/s, batched/mixed vs plain, at rel Frobenius err ≤1e-6"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


# HBM bytes per timed unit of a line, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# passes (KiB per dispatch of the line's kernels, summed over one unit),
# scaled by what the same counters read for a plain 1 GiB device copy
# (1 GiB read, 1 GiB written).  Each entry describes the kernels built from
# the listed sources with the SHA-1 given and is reported only while those
# sources still hash to it.  The summaries with the commands are under
# profiles/.
_CS = "paper_1710_07946_amd/csrc/"
SRC_TEAM = (_CS + "lra_ca.hip", _CS + "lra_common.h", _CS + "lra_device.h", _CS + "lra_internal.h",
            _CS + "lra_api.hip", "paper_1710_07946_amd/build.py")
SRC_BATCH = (_CS + "lra_batch.hip", _CS + "lra_common.h", _CS + "lra_device.h", _CS + "lra_internal.h",
             _CS + "lra_api.hip", "paper_1710_07946_amd/build.py")
SRC_POST = (_CS + "lra_post.hip", _CS + "lra_device.h", _CS + "lra_internal.h", "paper_1710_07946_amd/build.py")
SRC_DMM = (_CS + "lra_dmm.hip", _CS + "lra_common.h", _CS + "lra_device.h", _CS + "lra_internal.h",
           _CS + "lra_api.hip", "paper_1710_07946_amd/build.py")
# line: (sources, SHA-1, FETCH_SIZE KiB per unit, WRITE_SIZE KiB per unit, copy FETCH KiB, copy WRITE KiB)
TRAFFIC_COUNTS = {
    # one LRA: one ca_team_kernel dispatch (profiles/ca_team_kernel_20000x20000_r50.md)
    "headline": (SRC_TEAM, "ea7f432bf3c150ca12aaa4bc28419e1d07f89a3e", 324544.3, 108622.0, 524308.2, 1048576.0),
    # one batch: the four bin dispatches of ca_reg_kernel (profiles/ca_reg_kernel_fmm4096_r16.md)
    "batched": (SRC_BATCH, "178db4791ebf57fb8191e4168ef37c8e4eab14f2", 967.0 + 309103.3 + 3948961.9 + 7843.7, 38.0 + 1638.1 + 7639.3 + 313.5,
                524308.2, 1048576.0),
    # one batch: the four bin dispatches of ca_reg_points_kernel
    "points": (SRC_BATCH, "178db4791ebf57fb8191e4168ef37c8e4eab14f2", 815.6 + 4330.1 + 32443.1 + 1165.1, 38.0 + 1637.7 + 7643.0 + 313.5,
               524308.2, 1048576.0),
    # one full residual: the resid_kernel dispatch (FP64 core; BF16 x 3 core)
    # (profiles/resid_kernels_20000x20000_r50.md)
    "residual_fp64": (SRC_POST, "be83459b920890769ea07f68e587dfd02a3fed7b", 972149.4, 68.7, 524308.2, 1048576.0),
    "residual_mixed": (SRC_POST, "be83459b920890769ea07f68e587dfd02a3fed7b", 965536.3, 68.7, 524308.2, 1048576.0),
    # one launch of 256 blocks: the seven adj_* dispatches (profiles/adjoint_kernels_256x2048_r32.md)
    "adjoint": (SRC_POST, "be83459b920890769ea07f68e587dfd02a3fed7b", 1174708.3, 563418.4, 524308.2, 1048576.0),
    # one batch of 256 DMM08 C-A LRAs at k = l = 64: one ca_dmm_kernel dispatch
    # (profiles/ca_dmm_kernel_256x1000x1000_r16.md)
    "dmm_k64": (SRC_DMM, "937bf9044a9df50b72f0c2717eefc55621864995", 7496471.4, 72464.1, 524308.2, 1048576.0),
}


def sources_sha1(files):
    import hashlib
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_traffic(line):
    """Counter bytes per unit of `line`, or None once its kernels' sources changed."""
    src, sha, fetch, write, copy_fetch, copy_write = TRAFFIC_COUNTS[line]
    if sources_sha1(src) != sha:
        return None
    return 1024.0 * (fetch * (1048576.0 / copy_fetch) + write * (1048576.0 / copy_write))


def algorithmic_bytes(m, n, r, sweeps_run, depth, samples, elem):
    """Entries of A the LRA must read: 2^d rows (m >= n) or columns (m < n) per
    sampled multiplier column for the sketch, the seed row panel when the
    sketch picks rows (m < n), (m + n) r per sweep, the r x r generator."""
    if m >= n:
        cells = n * (2 ** depth) * samples + sweeps_run * (m * r + r * n) + r * r
    else:
        cells = m * (2 ** depth) * samples + r * n + sweeps_run * (m * r + r * n) + r * r
    return cells * elem


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="time only the headline LRA (skip batched, residual and adjoint lines)")
    ap.add_argument("--only", choices=["batched", "points", "cynical", "adjoint", "tall", "residual", "starts", "dmm"],
                    default=None,
                    help="time one secondary line alone and print it (for profiling)")
    ap.add_argument("--no-plain-loop", action="store_true",
                    help="batched line: skip the comparison loop of single-LRA launches")
    ap.add_argument("--save-sets", default=None,
                    help="residual / adjoint line: write the index sets of the forward C-A to this .npz")
    ap.add_argument("--sets", default=None,
                    help="residual / adjoint line: read the index sets from this .npz instead of running the "
                         "forward C-A (so a profiled run holds only the line's own kernels)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the C-A path is single-GPU; "
              "--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_ref_mib:
        src = torch.ones(args.copy_ref_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes": src.numel() * 4}))
        return

    import paper_1710_07946_amd as lra
    from paper_1710_07946_amd import workloads

    lra.load()
    if args.only in ("batched", "points", "cynical", "adjoint", "tall", "dmm"):
        fn = {"batched": bench_batched, "points": bench_points, "cynical": bench_cynical, "adjoint": bench_adjoint,
              "tall": bench_tall, "dmm": bench_dmm}[args.only]
        print(json.dumps({args.only: fn(lra, workloads, torch, np, args)}), flush=True)
        return
    t0 = time.time()
    A_np = workloads.factor_gaussian(M, N, RANK, 1e-6)
    print("# input generated in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    A = torch.from_numpy(A_np).cuda()
    kw = dict(preprocess=lra.LRA_PRE_ASRHT, ah_depth=DEPTH, ah_samples=SAMPLES)

    if args.only == "residual":
        if args.sets:
            z = np.load(args.sets)
            I, J = (torch.from_numpy(z[k]).cuda() for k in ("I", "J"))
            U = torch.from_numpy(z["U"]).cuda()
        else:
            out = lra.lra_cur(A, RANK, SWEEPS, SEED, **kw)
            I, J, U = out.I, out.J, out.U
            if args.save_sets:
                np.savez(args.save_sets, I=I.cpu().numpy(), J=J.cpu().numpy(), U=U.cpu().numpy())
        print(json.dumps({"residual": residual_fields(lra, torch, A, I, J, U, M, N, RANK, 4,
                                                      max(2, args.steps // 5))}), flush=True)
        return
    out = lra.lra_cur(A, RANK, SWEEPS, SEED, **kw)
    torch.cuda.synchronize()
    if args.only == "starts":
        print(json.dumps({"bidiag_start": bench_bidiag_start(lra, torch, np, A, args),
                          "fourier_start": bench_fourier_start(lra, torch, np, A, args),
                          "leverage_refinement": bench_leverage(lra, torch, np, A, args),
                          "preprocessed_ca": bench_preprocessed(lra, torch, np, A, args)}), flush=True)
        return
    for _ in range(args.warmup):
        lra.lra_cur(A, RANK, SWEEPS, SEED, out=out, **kw)
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        lra.lra_cur(A, RANK, SWEEPS, SEED, out=out, **kw)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    per = [starts[k].elapsed_time(ends[k]) for k in range(args.steps)]
    total_ms = starts[0].elapsed_time(ends[-1])
    ms_per_step = total_ms / args.steps
    kernel_ms = float(np.mean(per))
    info = out.info()
    if info["status"] != 0:
        raise SystemExit("lra_cur failed on the GPU: %s" % info)
    I, J, U = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy()

    resid = None if args.no_secondary else residual_fields(lra, torch, A, out.I, out.J, out.U, M, N, RANK, 4,
                                                          max(2, args.steps // 5))
    nbytes = algorithmic_bytes(M, N, RANK, info["sweeps_run"], DEPTH, SAMPLES, 4)
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    rec = {
        "metric": METRIC,
        "value": args.steps / (total_ms * 1e-3),
        "unit": "LRAs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "20000x20000 fp32 factor-Gaussian rank 50 + N(0,1e-6^2) noise; abridged SRHT "
                               "start (d=3, l=100); r=50, 4 sweeps, delta=0.01; FP64 panels and nucleus",
                   "m": M, "n": N, "r": RANK, "sweeps": SWEEPS, "ah_depth": DEPTH, "ah_samples": SAMPLES,
                   "seed": SEED, "input_dtype": "fp32"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counted_traffic("headline")},
        "useful_bytes_per_lra": nbytes,
        "kernel_ms": kernel_ms,
        "host_wall_ms_per_step": wall * 1e3 / args.steps,
        "team_size": info["team_size"],
        "sweeps_run": info["sweeps_run"],
        "swaps_total": info["swaps_total"],
    }

    # the decisions' smallest margin, from a run of the instantiation that
    # tracks it (outside the timed steps; its own time reported beside)
    mout = lra.lra_cur(A, RANK, SWEEPS, SEED, track_margin=True, **kw)
    ms_tracked = _time_events(torch, lambda: lra.lra_cur(A, RANK, SWEEPS, SEED, out=mout, track_margin=True, **kw),
                              max(2, args.steps // 5), 1)
    minfo = mout.info()
    rec["decision_margin"] = {"min_margin": minfo["min_margin"], "ms_per_lra_tracked": ms_tracked,
                              "sets_equal_untracked": bool(torch.equal(mout.I, out.I) and torch.equal(mout.J, out.J))}
    hop_ns = lra.lra_probe_exchange(20000)
    sel = selections_per_lra(M, N, RANK, info["sweeps_run"], info["swaps_total"], 1, SAMPLES)
    min_ms = sel * hop_ns * 1e-6
    rec["latency_roofline"] = {"bound": "cross-XCD exchange latency", "selections": sel, "hop_ns": hop_ns,
                               "min_ms": min_ms, "achieved_ms": kernel_ms, "frac": min_ms / kernel_ms}
    if not args.no_secondary:
        rec["hbm_stream_probe"] = hbm_stream_probe(torch)
    if resid is not None:
        rec["residual"] = resid
    if not args.no_cpu_baseline:
        import oracle
        times = []
        res = None
        t_all = time.perf_counter()
        while True:
            t1 = time.perf_counter()
            res = oracle.ca_cur(A_np, RANK, SWEEPS, SEED, preprocess=1, ah_depth=DEPTH, ah_samples=SAMPLES)
            times.append(time.perf_counter() - t1)
            if time.perf_counter() - t_all >= args.cpu_seconds:
                break
        rec["cpu_baseline"] = {"value": len(times) / sum(times), "unit": "LRAs/s", "cores": 1, "kind": "oracle",
                               "sample": "%d full LRAs of the same 20000x20000 workload, single-threaded FP64 oracle"
                                         % len(times), "host": host_info()}
        rows = np.sort(np.random.default_rng(0).choice(M, 400, replace=False))
        A64 = A_np[rows].astype(np.float64)
        Xo = A64[:, res.J] @ res.U @ A_np[res.I].astype(np.float64)
        Xg = A64[:, J] @ U @ A_np[I].astype(np.float64)
        rec["parity"] = {"sets_equal": bool(I.tolist() == res.I.tolist() and J.tolist() == res.J.tolist()),
                         "recon_rel_fro_diff_sampled": float(np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)),
                         "oracle_min_margin": res.min_margin,
                         "gpu_min_margin": minfo["min_margin"],
                         "rel_fro_err_vs_A_sampled": float(np.linalg.norm(A64 - Xg) / np.linalg.norm(A64))}
    if not args.no_secondary:
        rec["bidiag_start"] = bench_bidiag_start(lra, torch, np, A, args)
        rec["fourier_start"] = bench_fourier_start(lra, torch, np, A, args)
        rec["leverage_refinement"] = bench_leverage(lra, torch, np, A, args)
        rec["preprocessed_ca"] = bench_preprocessed(lra, torch, np, A, args)
        del A
        torch.cuda.empty_cache()
        rec["secondary"] = {
            "batched_fmm": bench_batched(lra, workloads, torch, np, args),
            "batched_fmm_points": bench_points(lra, workloads, torch, np, args),
            "adjoint_2048": bench_adjoint(lra, workloads, torch, np, args),
            "tall_65536x8192": bench_tall(lra, workloads, torch, np, args),
            "cynical_20000x20000_r16": bench_cynical(lra, workloads, torch, np, args),
            "dmm08_ca_1000x1000": bench_dmm(lra, workloads, torch, np, args),
        }
    if "hbm_stream_probe" in rec:
        add_attainable(rec, rec["hbm_stream_probe"]["copy_gbs"])
    print(json.dumps(rec), flush=True)


def add_attainable(node, copy_gbs):
    """Beside the 8 TB/s peak, every HBM roofline also states the bandwidth a
    plain device copy reached in the same run and its fraction of that."""
    if isinstance(node, dict):
        for key in ("roofline", "roofline_mixed"):
            rl = node.get(key)
            if isinstance(rl, dict) and rl.get("bound") == "hbm":
                rl["attainable"] = copy_gbs
                rl["frac_of_attainable"] = rl["achieved"] / copy_gbs
        for v in node.values():
            add_attainable(v, copy_gbs)


def bench_bidiag_start(lra, torch, np, A, args):
    """The headline matrix with the start set taken from the quasi-Gaussian
    multiplier of q = 3 random bidiagonal factors (l = 100 sampled columns)
    instead of the abridged SRHT; r = 50, 4 sweeps."""
    kw = dict(preprocess=lra.LRA_PRE_BIDIAG, ah_depth=3, ah_samples=SAMPLES)
    out = lra.lra_cur(A, RANK, SWEEPS, SEED, **kw)
    ms = _time_events(torch, lambda: lra.lra_cur(A, RANK, SWEEPS, SEED, out=out, **kw), max(2, args.steps // 5), 1)
    info = out.info()
    mom = lra.lra_residual(A, out.I, out.J, out.U).cpu().numpy()
    return {"workload": "headline matrix; start from QRP on W^T G_3 S (3 bidiagonal factors, l=100); r=50, 4 sweeps",
            "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"], "sweeps_run": info["sweeps_run"],
            "rel_fro_err": float(np.sqrt(mom[1] / mom[3]))}


def bench_fourier_start(lra, torch, np, A, args):
    """The headline matrix with the start set taken from the abridged
    randomized Fourier multiplier (d = 3, l = 50 complex columns, a real
    sketch of 100 columns as for the SRHT start); r = 50, 4 sweeps."""
    kw = dict(preprocess=lra.LRA_PRE_ASRFT, ah_depth=3, ah_samples=SAMPLES // 2)
    out = lra.lra_cur(A, RANK, SWEEPS, SEED, **kw)
    ms = _time_events(torch, lambda: lra.lra_cur(A, RANK, SWEEPS, SEED, out=out, **kw), max(2, args.steps // 5), 1)
    info = out.info()
    mom = lra.lra_residual(A, out.I, out.J, out.U).cpu().numpy()
    return {"workload": "headline matrix; start from QRP on the real form of the abridged SRFT sketch (d=3, "
                        "l=50 complex columns); r=50, 4 sweeps",
            "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"], "sweeps_run": info["sweeps_run"],
            "rel_fro_err": float(np.sqrt(mom[1] / mom[3]))}


def bench_leverage(lra, torch, np, A, args):
    """Refinement of the headline CUR by its leverage scores: k = l = 4r = 200
    rows and columns drawn by the scores of the r = 50 C-A CUR's own factors,
    U = D M_50^+ Dbar (the crude CUR from the headline call, not timed).
    4r is far below the sample sizes of Theorem thdmm (which grow with
    r^2 / eps^2); the line reports what it reaches."""
    base = lra.lra_cur(A, RANK, SWEEPS, SEED, preprocess=lra.LRA_PRE_ASRHT, ah_depth=3, ah_samples=SAMPLES)
    k = 4 * RANK
    out = lra.lra_cur_leverage(A, base.I, base.J, k, k, SEED)
    ms = _time_events(torch, lambda: lra.lra_cur_leverage(A, base.I, base.J, k, k, SEED, out=out),
                      max(2, args.steps // 5), 1)
    info = out.info()
    base_mom = lra.lra_residual(A, base.I, base.J, base.U).cpu().numpy()
    nbytes = 4 * (RANK * (M + N) + k * k)  # C and R read once, the generator
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"workload": "headline matrix; leverage scores of its r=50 C-A CUR's factors, k=l=200 draws (4r, "
                        "below the Theorem thdmm sample sizes), rank-50 canonical nucleus",
            "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"],
            "rel_fro_err": rel_err_k_by_l(torch, A, out.I, out.J, out.U),
            "crude_rel_fro_err": float(np.sqrt(base_mom[1] / base_mom[3])),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "traffic": None},
            "useful_bytes_per_lra": nbytes}


def rel_err_k_by_l(torch, A, I, J, U, rows=2000):
    """||W - W[:, J] U W[I, :]||_F / ||W||_F in FP64 by blocks of rows, for
    a k x l CUR beyond the residual kernel's square r <= 64 generators (an
    error check outside the timed region)."""
    R = A[I].to(torch.float64)
    CU = A[:, J].to(torch.float64) @ U
    e2 = w2 = 0.0
    for i0 in range(0, A.shape[0], rows):
        Wb = A[i0:i0 + rows].to(torch.float64)
        e2 += float(torch.linalg.norm(Wb - CU[i0:i0 + rows] @ R) ** 2)
        w2 += float(torch.linalg.norm(Wb) ** 2)
    return (e2 / w2) ** 0.5


def bench_preprocessed(lra, torch, np, A, args):
    """C-A on the pre-processed headline matrix W' = W D (H_8 (x) I_2500)
    (entries formed on the fly, r = 50, 4 sweeps).  Since M M^T = 8 I, the LRA
    of W is W'[:, J] U W[I, :]; its error is measured on 2000 sampled rows."""
    d = 3
    out = lra.lra_cur_hadamard(A, RANK, SWEEPS, SEED, d)
    ms = _time_events(torch, lambda: lra.lra_cur_hadamard(A, RANK, SWEEPS, SEED, d, out=out), max(2, args.steps // 5), 1)
    info = out.info()
    rows = torch.from_numpy(np.sort(np.random.default_rng(1).choice(M, 2000, replace=False))).cuda()
    W = A.to(torch.float64)
    q2, s = 1 << d, (N + (1 << d) - 1) >> d
    sgn = torch.from_numpy(np.array([oracle_free_sign(SEED, c) for c in range(N)])).cuda()
    Jh = out.J.cpu().numpy()
    cols = []
    for j in Jh:
        b, e = divmod(int(j), s)
        acc = torch.zeros(len(rows), dtype=torch.float64, device="cuda")
        for a in range(q2):
            c = a * s + e
            if c < N:
                h = -1.0 if bin(a & b).count("1") & 1 else 1.0
                acc += W[rows, c] * sgn[c] * h
        cols.append(acc)
    Cp = torch.stack(cols, 1)
    E = W[rows] - Cp @ out.U @ W[out.I]
    err = float(torch.linalg.norm(E) / torch.linalg.norm(W[rows]))
    return {"workload": "headline matrix pre-processed by D (H_8 kron I_2500), entries on the fly; r=50, 4 sweeps",
            "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"], "team_size": info["team_size"],
            "sweeps_run": info["sweeps_run"], "rel_fro_err_sampled_2000_rows": err}


def oracle_free_sign(seed, c):
    """The Rademacher sign of column c (SplitMix64 stream 1, the multiplier's D), for the error check."""
    mask = (1 << 64) - 1
    z = (seed + 0x9E3779B97F4A7C15 * ((1 << 40) + c + 1)) & mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    z ^= z >> 31
    return -1.0 if z >> 63 else 1.0


def host_info():
    """Host cores and CPU model, for the CPU baselines."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def oracle_rate(jobs, threads, seconds):
    """Run oracle jobs (callables) on `threads` host threads (the oracle's
    calls release the interpreter lock) for about `seconds`, or until the
    list is used up; returns (jobs done, wall seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    done = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for i in range(0, len(jobs), threads):
            list(ex.map(lambda f: f(), jobs[i:i + threads]))
            done += len(jobs[i:i + threads])
            if time.perf_counter() - t0 >= seconds:
                break
    return done, time.perf_counter() - t0


def hbm_stream_probe(torch):
    """Attainable HBM bandwidth from torch kernels on 2 GiB: a device-to-device
    copy (read + write) and a sum (read)."""
    x = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    nbytes = x.numel() * 4
    ms_copy = _time_events(torch, lambda: y.copy_(x), 10, 2)
    ms_sum = _time_events(torch, lambda: x.sum(), 10, 2)
    del x, y
    torch.cuda.empty_cache()
    return {"copy_gbs": 2 * nbytes / (ms_copy * 1e-3) / 1e9, "read_gbs": nbytes / (ms_sum * 1e-3) / 1e9,
            "bytes": nbytes, "kernels": "torch copy_ and sum on 2 GiB fp32"}


def selections_per_lra(m, n, r, sweeps_run, swaps_total, pre, samples):
    """Team-wide decisions of one LRA: r QRP pivots of the sketch start, r LU
    pivots and one stop test per step (2 per sweep, plus the seed row step
    when the sketch picks rows), and one per swap."""
    steps = 2 * sweeps_run + (1 if (pre and m < n) else 0)
    return (r if pre else 0) + steps * (r + 1) + swaps_total


def _time_events(torch, fn, steps, warmup):
    """Mean milliseconds of fn() over `steps` calls, HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def residual_fields(lra, torch, A, I, J, U, m, n, r, elem, steps):
    """Full residual moments of a computed CUR in FP64 (FP64 matrix cores) and
    in mixed precision (BF16 x 3 matrix cores, FP32 accumulation), plus the
    sampled 256 x 256 estimate, each timed."""
    mom = torch.empty(4, dtype=torch.float64, device=A.device)
    ms_full = _time_events(torch, lambda: lra.lra_residual(A, I, J, U, out=mom), steps, 1)
    full = mom.cpu().numpy()
    ms_mixed = _time_events(torch, lambda: lra.lra_residual(A, I, J, U, prec=lra.LRA_PREC_MIXED, out=mom), steps, 1)
    mixed = mom.cpu().numpy()
    ms_samp = _time_events(torch, lambda: lra.lra_residual(A, I, J, U, 256, 256, 7, out=mom), steps, 1)
    samp = mom.cpu().numpy()
    flops = 2.0 * m * n * r + 2.0 * r * r * n
    tflops = flops / (ms_full * 1e-3) / 1e12
    gbs_mixed = m * n * elem / (ms_mixed * 1e-3) / 1e9
    err_full = math.sqrt(full[1] / full[3])
    # counter bytes describe the 20000 x 20000 FP32 headline matrix only
    headline = (m, n, r, elem) == (M, N, RANK, 4)
    traffic_fp64 = counted_traffic("residual_fp64") if headline else None
    traffic_mixed = counted_traffic("residual_mixed") if headline else None
    err_mixed = math.sqrt(mixed[1] / mixed[3])
    return {
        "ms_full_fp64": ms_full, "ms_full_mixed": ms_mixed, "ms_sampled_256x256": ms_samp,
        "rel_fro_err_full_fp64": err_full,
        "rel_fro_err_full_mixed": err_mixed,
        "mixed_vs_fp64_rel_diff_of_err": abs(err_mixed - err_full) / err_full,
        "rel_fro_err_sampled_256x256": float(math.sqrt(samp[1] / samp[3])),
        "roofline_fp64": {"bound": "mfma", "achieved": tflops, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                          "frac": tflops / FP64_PEAK_TFS, "traffic": traffic_fp64},
        "roofline_mixed": {"bound": "hbm", "achieved": gbs_mixed, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs_mixed / HBM_PEAK_GBS, "traffic": traffic_mixed},
    }


def bench_batched(lra, workloads, torch, np, args):
    """4096 FMM far-field blocks (rows, columns uniform in 64..1024), r = 16,
    3 sweeps: one persistent launch against a loop of single-LRA launches."""
    count, r, sweeps, seed = 4096, 16, 3, 1000
    t0 = time.time()
    base, desc = workloads.fmm_batch_device(count, "cuda")
    torch.cuda.synchronize()
    print("# fmm blocks generated in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    out = lra.lra_cur_batched(base, desc, r, sweeps, seed)
    ms = _time_events(torch, lambda: lra.lra_cur_batched(base, desc, r, sweeps, seed, out=out),
                      max(2, args.steps // 5), 1)
    infos = out.info()
    bad = [i for i in infos if i["status"] != 0]
    nbytes = sum(4 * (inf["sweeps_run"] * (int(d[1]) * r + r * int(d[2])) + r * r) for inf, d in zip(infos, desc))
    sector_bytes = sum(inf["sweeps_run"] * (64 * int(d[1]) * min(r, -(-int(d[2]) // 16)) + 4 * r * int(d[2]))
                       + 64 * r * r for inf, d in zip(infos, desc))
    loop_n = 256
    ms_loop, same = float("nan"), None
    if not args.no_plain_loop:
        views = [base[int(d[0]):int(d[0]) + int(d[1]) * int(d[2])].view(int(d[1]), int(d[2])) for d in desc[:loop_n]]
        outs = [lra.lra_cur(views[b], r, sweeps, seed + b) for b in range(loop_n)]

        def loop():
            for b in range(loop_n):
                lra.lra_cur(views[b], r, sweeps, seed + b, out=outs[b])

        ms_loop = _time_events(torch, loop, 2, 1)
        same = all(outs[b].I.cpu().tolist() == out.I[b].cpu().tolist() and
                   outs[b].J.cpu().tolist() == out.J[b].cpu().tolist() for b in range(8))
        del outs, views
    gbs = nbytes / (ms * 1e-3) / 1e9
    res = {
        "workload": "4096 FMM blocks 1/|x-y|, m, n uniform in 64..1024, fp32; r=16, 3 sweeps, random start",
        "lras_per_s": count / (ms * 1e-3), "ms_per_batch": ms,
        "plain_loop_lras_per_s": None if args.no_plain_loop else loop_n / (ms_loop * 1e-3),
        "plain_loop_sample": "first %d blocks" % loop_n,
        "speedup_vs_plain_loop": None if args.no_plain_loop else (count / ms) / (loop_n / ms_loop),
        "failed_blocks": len(bad), "first_8_match_plain_calls": same,
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": counted_traffic("batched")},
        "useful_bytes_per_batch": nbytes,
        # a strided FP32 column entry moves at least one 64-byte sector
        "sector_bytes_per_batch": sector_bytes,
        "bin_rules": [list(q) for q in lra.lra_batch_get_rules()],
    }
    if not args.no_cpu_baseline:
        import oracle
        hostbuf = base.cpu().numpy()

        def job(b):
            o0, m, n = int(desc[b][0]), int(desc[b][1]), int(desc[b][2])
            return lambda: oracle.ca_cur(hostbuf[o0:o0 + m * n].reshape(m, n), r, sweeps, seed + b)

        nth = os.cpu_count() or 1
        d1, t1 = oracle_rate([job(b) for b in range(0, count, 97)], 1, args.cpu_seconds / 2)
        dn, tn = oracle_rate([job(b) for b in range(count)], nth, args.cpu_seconds / 2)
        res["cpu_baseline"] = {"value": dn / tn, "unit": "LRAs/s", "cores": nth, "kind": "oracle",
                               "value_1_core": d1 / t1,
                               "sample": "%d blocks on %d threads, %d blocks on 1 thread (blocks in index order, "
                                         "sizes as in the batch)" % (dn, nth, d1),
                               "host": host_info()}
    # the same blocks by CUR with uniform leverage scores (k = l = 4r = 64
    # rows and columns drawn with replacement, rank-16 canonical nucleus):
    # only the 64 x 64 generator of each block is read
    k = 64
    uo = lra.lra_cur_uniform_batched(base, desc, r, k, k, seed)
    ms_u = _time_events(torch, lambda: lra.lra_cur_uniform_batched(base, desc, r, k, k, seed, out=uo),
                        max(2, args.steps // 5), 1)
    uinfos = uo.info()

    def rel_err(b, I, J, U):
        o0, m, n = int(desc[b][0]), int(desc[b][1]), int(desc[b][2])
        blk = base[o0:o0 + m * n].view(m, n).double()
        E = blk - blk[:, J] @ U @ blk[I]
        return float(torch.linalg.norm(E) / torch.linalg.norm(blk))

    sample = range(0, count, count // 8)
    errs_u = [rel_err(b, uo.I[b], uo.J[b], uo.U[b]) for b in sample]
    errs_ca = [rel_err(b, out.I[b], out.J[b], out.U[b]) for b in sample]
    nbytes_u = count * 4 * k * k
    gbs_u = nbytes_u / (ms_u * 1e-3) / 1e9
    res["uniform_leverage_k64_l64"] = {
        "lras_per_s": count / (ms_u * 1e-3), "ms_per_batch": ms_u,
        "failed_blocks": sum(1 for i in uinfos if i["status"] != 0),
        "median_rel_fro_err_8_blocks": float(np.median(errs_u)),
        "ca_median_rel_fro_err_same_blocks": float(np.median(errs_ca)),
        "roofline": {"bound": "hbm", "achieved": gbs_u, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs_u / HBM_PEAK_GBS, "traffic": None},
        "useful_bytes_per_batch": nbytes_u,
    }
    del base, out, uo
    torch.cuda.empty_cache()
    return res


def bench_points(lra, workloads, torch, np, args):
    """The same 4096 FMM far-field blocks given by their point sets, every entry
    K_ij = 1/|x_i - y_j| evaluated on the fly in FP64 (no block is stored),
    r = 16, 3 sweeps, one persistent launch."""
    count, r, sweeps, seed = 4096, 16, 3, 1000
    pts_np, desc = workloads.fmm_points(count)
    pts = torch.from_numpy(pts_np).cuda()
    out = lra.lra_cur_batched_points(pts, desc, r, sweeps, seed)
    ms = _time_events(torch, lambda: lra.lra_cur_batched_points(pts, desc, r, sweeps, seed, out=out),
                      max(2, args.steps // 5), 1)
    infos = out.info()
    bad = [i for i in infos if i["status"] != 0]
    # entries formed: each sweep's column and row panels, plus the generator
    entries = sum(inf["sweeps_run"] * (int(d[2]) * r + r * int(d[3])) + r * r for inf, d in zip(infos, desc))
    flops = 7.0 * entries  # 2 subtractions, 2 products, 1 sum, 1 square root, 1 division per entry
    tfs = flops / (ms * 1e-3) / 1e12
    res = {
        "workload": "4096 FMM blocks 1/|x-y| from their point sets (m, n uniform in 64..1024), entries formed "
                    "on the fly in fp64; r=16, 3 sweeps, random start",
        "lras_per_s": count / (ms * 1e-3), "ms_per_batch": ms, "failed_blocks": len(bad),
        "entries_per_batch": entries, "point_bytes": int(pts_np.nbytes),
        "roofline": {"bound": "alu", "achieved": tfs, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": tfs / FP64_PEAK_TFS, "traffic": counted_traffic("points")},
    }
    del pts, out
    torch.cuda.empty_cache()
    return res


def bench_adjoint(lra, workloads, torch, np, args):
    """256 blocks of 2048 x 2048 FP32 rank-32 factor products + N(0, 1e-5^2);
    index sets from a forward C-A at r = 32 (3 sweeps); loss on 1% of the
    entries; time of one adjoint launch over all blocks."""
    count, m, n, r, nnz = 256, 2048, 2048, 32, 41943
    t0 = time.time()
    Cs, Rs, Gs, rows, cols, vals = [], [], [], [], [], []
    g = torch.Generator(device="cuda")
    g.manual_seed(4242)
    sets = np.load(args.sets) if args.sets else None
    saved_I, saved_J = [], []
    for b in range(count):
        A = workloads.factor_gaussian_device(m, n, r, 1e-5, 6000 + b, "cuda")
        if sets is not None:
            Ib, Jb = torch.from_numpy(sets["I"][b]).cuda(), torch.from_numpy(sets["J"][b]).cuda()
        else:
            res = lra.lra_cur(A, r, 3, 7000 + b)
            Ib, Jb = res.I, res.J
            saved_I.append(Ib.cpu().numpy())
            saved_J.append(Jb.cpu().numpy())
        A64 = A.to(torch.float64)
        Cs.append(A64[:, Jb])
        Rs.append(A64[Ib])
        Gs.append(A64[Ib][:, Jb])
        flat = torch.sort(torch.randperm(m * n, generator=g, device="cuda")[:nnz]).values
        rows.append((flat // n).to(torch.int32))
        cols.append((flat % n).to(torch.int32))
        vals.append(A64.reshape(-1)[flat])
    if args.save_sets and sets is None:
        np.savez(args.save_sets, I=np.stack(saved_I), J=np.stack(saved_J))
    C, R, G = (torch.stack(x).contiguous() for x in (Cs, Rs, Gs))
    om_row, om_col, a_om = (torch.stack(x).contiguous() for x in (rows, cols, vals))
    order = lra.omega_column_order(om_row, om_col)
    torch.cuda.synchronize()
    print("# adjoint inputs prepared in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    out = {}

    def run():
        out["r"] = lra.lra_cur_adjoint(C, R, G, om_row, om_col, order, a_om)

    ms = _time_events(torch, run, max(2, args.steps // 2), 1)
    st = out["r"][4]
    nbytes = count * (2 * 8 * (m * r + r * n + r * r) + nnz * (4 + 4 + 4 + 8))
    gbs = nbytes / (ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nth = os.cpu_count() or 1
        sample = min(count, 2 * nth)
        host = [(C[b].cpu().numpy(), R[b].cpu().numpy(), G[b].cpu().numpy(), om_row[b].cpu().numpy(),
                 om_col[b].cpu().numpy(), a_om[b].cpu().numpy()) for b in range(sample)]
        jobs = [(lambda h=h: oracle.cur_adjoint(*h)) for h in host]
        d1, t1 = oracle_rate(jobs[:2], 1, args.cpu_seconds / 2)
        dn, tn = oracle_rate(jobs, nth, args.cpu_seconds / 2)
        cpu = {"value": dn / tn, "unit": "blocks/s", "cores": nth, "kind": "oracle", "value_1_core": d1 / t1,
               "sample": "%d blocks on %d threads, %d on 1 thread (FP64 analytic loss and gradients)"
                         % (dn, nth, d1), "host": host_info()}
    return {
        "cpu_baseline": cpu,
        "workload": "256 blocks 2048x2048 fp32 rank-32 + N(0,1e-5^2), r=32, |Omega|=41943 per block, FP64",
        "blocks_per_s": count / (ms * 1e-3), "ms_per_launch": ms,
        "failed_blocks": int((st != 0).sum().item()),
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": counted_traffic("adjoint")},
        "useful_bytes_per_launch": nbytes,
    }


def bench_dmm(lra, workloads, torch, np, args):
    """C-A with DMM08 leverage-score sampling of every sketch (the C-A tests
    of Tables 7 and 8: 1000 x 1000 inputs of low numerical rank, eight
    iterations, k = l = 4r, 2r, r) on 256 blocks 1000 x 1000 FP32 of
    numerical rank 16 (graded Gaussian factors + N(0, 1e-6^2)), one launch
    per k; r = 16.  The k = l = 64 launch is the line's figure."""
    count, m, n, r, iters, seed = 256, 1000, 1000, 16, 8, 3000
    t0 = time.time()
    base, desc = workloads.graded_lowrank_batch_device(count, m, n, r, 1e-6, 8000, "cuda")
    torch.cuda.synchronize()
    print("# dmm blocks generated in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    res = {"workload": "256 blocks 1000x1000 fp32, X diag(10^(-2a/15)) Y + N(0,1e-6^2) (numerical rank 16); "
                       "r=16, 8 iterations of DMM08 row / column sampling on the sketches; k=l in {64, 32, 16}"}
    host = None
    for k in (64, 32, 16):
        out = lra.lra_cur_dmm_batched(base, desc, r, k, k, iters, seed)
        ms = _time_events(torch, lambda: lra.lra_cur_dmm_batched(base, desc, r, k, k, iters, seed, out=out),
                          max(2, args.steps // 10), 1)
        infos = out.info()
        I, J, U = out.I.cpu().numpy(), out.J.cpu().numpy(), out.U.cpu().numpy()
        if host is None:
            host = base[:8 * m * n].cpu().numpy().reshape(8, m, n).astype(np.float64)
        errs = []
        for b in range(8):
            X = host[b][:, J[b]] @ U[b] @ host[b][I[b]]
            errs.append(float(np.linalg.norm(host[b] - X) / np.linalg.norm(host[b])))
        # FP64 flops on the matrix cores per LRA: the Gram matrix (2 items w^2)
        # and the projections (2 items w r) of each half-step
        flops = count * iters * (2.0 * m * k * k + 2.0 * m * k * r + 2.0 * n * k * k + 2.0 * n * k * r)
        tfs = flops / (ms * 1e-3) / 1e12
        line = {"lras_per_s": count / (ms * 1e-3), "ms_per_batch": ms,
                "failed_blocks": sum(1 for i in infos if i["status"] != 0),
                "median_rel_fro_err_8_blocks": float(np.median(errs))}
        if k == 64:
            line["roofline"] = {"bound": "mfma", "achieved": tfs, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                                "frac": tfs / FP64_PEAK_TFS, "traffic": counted_traffic("dmm_k64")}
            line["useful_bytes_per_batch"] = count * (iters * 2 * (m * k + k * n) * 4 + k * k * 4)
        res["k%d" % k] = line
    if not args.no_cpu_baseline:
        import oracle
        nth = os.cpu_count() or 1
        jobs = [(lambda b=b: oracle.dmm_ca(host[b].astype(np.float32), r, 64, 64, iters, seed + b))
                for b in range(8)]
        d1, t1 = oracle_rate(jobs[:2], 1, args.cpu_seconds / 2)
        dn, tn = oracle_rate(jobs, nth, args.cpu_seconds / 2)
        res["cpu_baseline"] = {"value": dn / tn, "unit": "LRAs/s", "cores": nth, "kind": "oracle",
                               "value_1_core": d1 / t1,
                               "sample": "%d blocks (k=l=64) on %d threads, %d on 1 thread" % (dn, nth, d1),
                               "host": host_info()}
    del base
    torch.cuda.empty_cache()
    return res


def bench_cynical(lra, workloads, torch, np, args):
    """Cynical CUR on a 20000 x 20000 FP32 factor-Gaussian rank-16 input
    (+ N(0, 1e-6^2)): Tests 4 (one C-A loop at rank k = 4r = 64, then the
    r x r generator inside the 64 x 64 sketch) and Tests 3 (random 64 x 64
    sketch), beside plain C-A at r = 16 (4 sweeps) and C-A with 64 x 64
    generators of large 16-projective volume (3 sweeps); relative Frobenius
    errors from the FP64 residual."""
    m = n = 20000
    r, k = 16, 64
    A = workloads.factor_gaussian_device(m, n, r, 1e-6, 3011, "cuda")
    reps = max(2, args.steps // 5)
    rec = {"workload": "20000x20000 fp32 factor-Gaussian rank 16 + N(0,1e-6^2); r=16, k=l=64"}

    def err(out):
        mom = lra.lra_residual(A, out.I, out.J, out.U).cpu().numpy()
        return float(np.sqrt(mom[1] / mom[3]))

    for name, loops in (("tests4_one_loop", 1), ("tests3_random_sketch", 0)):
        out = lra.lra_cur_cynical(A, r, k, loops, 3, 2031)
        ms = _time_events(torch, lambda: lra.lra_cur_cynical(A, r, k, loops, 3, 2031, out=out), reps, 1)
        info = out.info()
        nbytes = 4 * (loops * (m + n) * k + k * k + r * r)
        gbs = nbytes / (ms * 1e-3) / 1e9
        rec[name] = {"lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"],
                     "team_size": info["team_size"], "rel_fro_err": err(out),
                     "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": gbs / HBM_PEAK_GBS, "traffic": None},
                     "useful_bytes_per_lra": nbytes}
    out = lra.lra_cur(A, r, 4, 2031)
    ms = _time_events(torch, lambda: lra.lra_cur(A, r, 4, 2031, out=out), reps, 1)
    rec["plain_ca_r16_4_sweeps"] = {"lras_per_s": 1e3 / ms, "ms_per_lra": ms, "rel_fro_err": err(out)}
    # refinement by leverage scores of a crude one-sweep C-A CUR, k = l = 4r
    crude = lra.lra_cur(A, r, 1, 2031)
    lev = lra.lra_cur_leverage(A, crude.I, crude.J, k, k, 2031)
    ms = _time_events(torch, lambda: lra.lra_cur_leverage(A, crude.I, crude.J, k, k, 2031, out=lev), reps, 1)
    info = lev.info()
    rec["leverage_refinement_of_1_sweep_ca_k64_l64"] = {
        "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"], "nucleus_rank": info["nucleus_rank"],
        "rel_fro_err": err(lev), "crude_rel_fro_err": err(crude)}
    # k x l = 64 x 64 generators of large r-projective volume, canonical
    # nucleus (U is l x k, so the r x r residual kernel takes it at rank 64)
    out = lra.lra_cur_projective(A, r, k, k, 3, 2031)
    ms = _time_events(torch, lambda: lra.lra_cur_projective(A, r, k, k, 3, 2031, out=out), reps, 1)
    info = out.info()
    nbytes = 4 * (info["sweeps_run"] * (m + n) * k + k * k)
    gbs = nbytes / (ms * 1e-3) / 1e9
    rec["projective_volume_k64_l64_3_sweeps"] = {
        "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"], "team_size": info["team_size"],
        "sweeps_run": info["sweeps_run"], "swaps_total": info["swaps_total"], "nucleus_rank": info["nucleus_rank"],
        "rel_fro_err": err(out),
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None},
        "useful_bytes_per_lra": nbytes}
    del A
    torch.cuda.empty_cache()
    return rec


def bench_tall(lra, workloads, torch, np, args):
    """65536 x 8192 FP32 of numerical rank 64 (Gaussian factors, unit singular
    values then i^-2 decay floored at 1e-7): left-form abridged SRHT start
    (d = 3, l = 128), r = 64, 4 sweeps, nucleus with two refinement steps;
    then the full residual in FP64 and in mixed precision."""
    m, n, r = 65536, 8192, 64
    t0 = time.time()
    A = workloads.decaying_spectrum_device(m, n, r, 1e-7, 1031, "cuda")
    torch.cuda.synchronize()
    print("# tall input generated in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    kw = dict(preprocess=lra.LRA_PRE_ASRHT, ah_depth=3, ah_samples=128, refine_steps=2)
    out = lra.lra_cur(A, r, 4, 2051, **kw)
    ms = _time_events(torch, lambda: lra.lra_cur(A, r, 4, 2051, out=out, **kw), max(2, args.steps // 5), 1)
    info = out.info()
    nbytes = algorithmic_bytes(m, n, r, info["sweeps_run"], 3, 128, 4)
    res = residual_fields(lra, torch, A, out.I, out.J, out.U, m, n, r, 4, max(2, args.steps // 5))
    gbs = nbytes / (ms * 1e-3) / 1e9
    rec = {
        "workload": "65536x8192 fp32, numerical rank 64 (Gaussian factors, sigma_i = 1 then i^-2, floor 1e-7); "
                    "left-form abridged SRHT d=3 l=128; r=64, 4 sweeps, nucleus with 2 refinement steps",
        "lras_per_s": 1e3 / ms, "ms_per_lra": ms, "status": info["status"], "team_size": info["team_size"],
        "sweeps_run": info["sweeps_run"],
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None},
        "useful_bytes_per_lra": nbytes,
        "residual": res,
    }
    del A
    torch.cuda.empty_cache()
    return rec


if __name__ == "__main__":
    main()
