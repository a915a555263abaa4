#!/usr/bin/env python3
"""Single-GPU benchmark of the single-pass PCA hot path (Algorithm 4) on MI355X.

Workload (FP32-resident): A is 100000 x 20000 FP32 (8.0 GB) resident in HBM, sigma_j = 1/j for
j <= 200 then 1e-4, with N(0, 1e-4) noise on sigma; k = 50, l = 100, b = 10; 25 row blocks of 4096
rows (the last 1696).  A is generated on the GPU from a Kronecker-structured SVD whose spectrum is
exactly known.  One step = one whole pass of the hot path: a new Omega from a seed (step 3), all
row blocks ingested (steps 4-8), and the finalize (steps 9-19) returning S, V.

The JSON line reports the headline mode (BF16 by default) and, under "compare", the FP32 mode,
each as FP32-equivalent ingest GB/s (4 m n bytes per step / step time).  Accuracy of each mode is
measured against the FP64 reference on the same stored A and the same Omega' (relative sigma_k
error; the gate is 1e-3).  The reference also provides the CPU baseline, timed on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A-ingest GB/s + % roofline, BF16 vs FP32 @ rel σ_k err≤1e-3; p99 block lat"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "bf16x2": 2500.0, "fp8": 5000.0, "f64": 78.6}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="fp32-resident",
                    choices=["fp32-resident", "host-c3", "host-c5"])
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="bf16", choices=["f32", "bf16", "bf16x2", "fp8", "f64"])
    ap.add_argument("--compare", default="f32,f64",
                    help="further modes reported alongside, comma-separated ('none' = none)")
    ap.add_argument("--m", type=int, default=100000)
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--kron", default="500,200,100,200", help="m1,m2,n1,n2 with m=m1*m2, n=n1*n2")
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--l", type=int, default=100)
    ap.add_argument("--b", type=int, default=0,
                    help="column block width of the finalize loop; 0 = l (one block, fastest)")
    ap.add_argument("--block", type=int, default=4096)
    ap.add_argument("--check", default="full", choices=["full", "none"],
                    help="FP64 reference accuracy check on the whole workload")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the CPU-baseline sample (0 = skip)")
    ap.add_argument("--serving-streams", type=int, default=64,
                    help="streams of the serving scenario (0 = skip it)")
    ap.add_argument("--serving-rho", type=float, default=0.8,
                    help="offered load of the Poisson phase, as a fraction of saturation")
    ap.add_argument("--serving-modes", default="f32,bf16")
    ap.add_argument("--serving-host", type=int, default=1,
                    help="1: also serve the streams from pinned host memory (first serving mode)")
    ap.add_argument("--power", default="bf16",
                    help="modes run with the power scheme P = 1 on the resident workload ('' = none)")
    ap.add_argument("--study", type=int, default=1,
                    help="1: the Sec. 4.1 accuracy study (Types 1-5, 3000 x 3000, every mode)")
    ap.add_argument("--host-configs", default="c5,c3",
                    help="host-streamed workloads also run by the default workload ('' = none)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (known bytes) to scale HBM "
                         "counters")
    return ap.parse_args()


def make_matrix(args, torch):
    import synth
    m1, m2, n1, n2 = (int(x) for x in args.kron.split(","))
    assert m1 * m2 == args.m and n1 * n2 == args.n, "--kron must factor m and n"
    sig = synth.noisy_spectrum(synth.inv_floor_spectrum(args.n, knee=200, floor=1e-4), 1e-4, 1002)
    K = synth.KronMatrix(m1, m2, n1, n2, sig, 1002)
    A = torch.empty(args.m, args.n, dtype=torch.float32, device="cuda")
    for r0 in range(0, args.m, 2048):
        c = min(2048, args.m - r0)
        K.rows_torch(r0, c, "cuda", out=A[r0:r0 + c])
    torch.cuda.synchronize()
    return A, K


def run_step(sk_obj, A, block, seed):
    sk_obj.reset(seed)
    m = A.shape[0]
    for r0 in range(0, m, block):
        sk_obj.ingest(A[r0:r0 + block])
    return sk_obj.finalize(want_u=False)


def bench_mode(mode, A, args, torch, sk):
    m, n = A.shape
    obj = sk.Sketch(n, m, args.block, args.k, args.l, args.b, compute=mode, seed=2002)
    for _ in range(args.warmup):
        run_step(obj, A, args.block, 2002)
    torch.cuda.synchronize()
    # per-kernel durations of the timed steps themselves: the library records HIP events on its
    # launch stream around each product and around the finalize
    obj.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S, V, _, rank = run_step(obj, A, args.block, 2002)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / max(1, args.steps)
    n1, t_g1 = obj.profile_read(0)
    n2, t_g2 = obj.profile_read(1)
    nf, t_fin = obj.profile_read(2)
    obj.profile(False)
    nblocks = (m + args.block - 1) // args.block
    res = dict(mode=mode, ms_per_step=ms_step, value=4.0 * m * n / (ms_step * 1e-3) / 1e9,
               rank=rank, S=S.cpu().numpy(), V=V.cpu().numpy(),
               gemm1_ms=t_g1 / max(1, n1), gemm2_ms=t_g2 / max(1, n2),
               finalize_ms=t_fin / max(1, nf), launches=(n1, n2, nf), nblocks=nblocks)
    obj.close()
    return res


def block_latency(A, args, torch, sk, mode):
    """Per-block ingest latency (enqueue to completion of that block's kernels), one block at a
    time, on the resident workload."""
    m, n = A.shape
    obj = sk.Sketch(n, m, args.block, args.k, args.l, args.b, compute=mode, seed=7)
    lat = []
    for r0 in range(0, m, args.block):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        obj.ingest(A[r0:r0 + args.block])
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    obj.close()
    full = [x for i, x in enumerate(lat) if (i + 1) * args.block <= m] or lat
    return float(np.percentile(full, 50)), float(np.percentile(full, 99))


def serving_bench(args, torch, sk, mode, host_too=False):
    """64 concurrent streams (n uniform over the multiples of 1024 up to 32768, m uniform in
    [10000, 200000] rows, sigma_j = exp(-j/20) for j <= 256 and 0 beyond; k = 20, l = 40, b = 10;
    blocks uniform in [256, 4096] rows), each a stacked pool resident on the GPU.

    Phase 1 submits every block of every stream at once and measures the saturated grouped
    throughput X.  Phase 2 replays the streams with per-stream Poisson block arrivals whose total
    offered load is rho X (each stream's byte rate proportional to its size, so all streams span
    the same interval), finalizing each stream on a helper thread when its last block has
    completed; the per-block latency (submit to completion) is reported as p50 / p99."""
    import threading
    import synth
    nstr = args.serving_streams
    draws = synth.draw_serving_streams(nstr, seed=30000)
    sig = np.zeros(1024)
    sig[:256] = np.exp(-np.arange(1, 257) / 20.0)
    pools = []
    for s_ in range(nstr):
        n, m = int(draws.n[s_]), int(draws.m[s_])
        pools.append(synth.serving_pool_torch(n, sig, m // 1024, 10000 + s_, "cuda"))
    torch.cuda.synchronize()
    k, l, b = 20, 40, 10
    probe = sk.Server(l, 32768, int(draws.m.max()), 4096, 0, compute=mode, src="f32", worker=False)
    foot = [probe.stream_bytes(int(draws.n[s_]), int(draws.m[s_]), k, b) for s_ in range(nstr)]
    probe.close()
    budget = int(sum(foot) * 1.05) + (64 << 20)
    total_bytes = float(sum(4.0 * int(draws.m[s_]) * int(draws.n[s_]) for s_ in range(nstr)))

    def blocks_of(s_, host=None):
        r0, out = 0, []
        pool = (host or pools)[s_]
        for rows in draws.blocks[s_]:
            a = r0 % 1024
            out.append(pool[a:a + int(rows)])
            r0 += int(rows)
        return out

    def run(arrivals, state_budget=None, opens=None, host=None):
        srv = sk.Server(l, 32768, int(draws.m.max()), 4096, state_budget or budget, compute=mode,
                        src="f32", max_group=16, worker=True, host_slots=4 if host else 0)
        sids = [None] * nstr
        if opens is None:
            for s_ in range(nstr):
                sids[s_] = srv.open(int(draws.n[s_]), int(draws.m[s_]), k, b, 20000 + s_)[0]
        events = []
        for s_ in range(nstr):
            if opens is not None:
                events.append((opens[s_], s_, -1, None))        # the stream request itself
            for i, blk in enumerate(blocks_of(s_, host)):
                events.append((0.0 if arrivals is None else arrivals[s_][i], s_, i, blk))
        events.sort(key=lambda e: (e[0], e[1], e[2]))
        last_tk = {}
        owner = {}
        lat = {}
        results = {}
        fin_threads = []
        remaining = {s_: len(draws.blocks[s_]) for s_ in range(nstr)}

        def fin(s_):
            S, V, _, rank = srv.finalize(sids[s_])
            results[s_] = (S.cpu().numpy(), rank)

        def drain():
            for tk, lt in srv.poll():
                lat[tk] = lt
                s_ = owner[tk]
                remaining[s_] -= 1
                if remaining[s_] == 0:
                    t = threading.Thread(target=fin, args=(s_,))
                    t.start()
                    fin_threads.append(t)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for at, s_, i, blk in events:
            while True:
                now = time.perf_counter() - t0
                if now >= at:
                    break
                drain()
                if at - now > 2e-4:
                    time.sleep(min(at - now, 1e-3) * 0.5)
            if i < 0:
                sids[s_] = srv.open(int(draws.n[s_]), int(draws.m[s_]), k, b, 20000 + s_)[0]
                continue
            tk = srv.submit(sids[s_], blk)
            owner[tk] = s_
            last_tk[s_] = tk
        nblk = sum(1 for e in events if e[2] >= 0)
        while len(lat) < nblk:
            drain()
            time.sleep(1e-4)
        t_pass = time.perf_counter() - t0
        for t in fin_threads:
            t.join()
        t_all = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lats = np.array(list(lat.values())) * 1e3
        errs = [abs(results[s_][0][k - 1] - sig[k - 1]) / sig[k - 1] for s_ in results]
        return dict(pass_s=t_pass, total_s=t_all, gbps=total_bytes / t_pass / 1e9,
                    p50_ms=float(np.percentile(lats, 50)), p99_ms=float(np.percentile(lats, 99)),
                    blocks=int(st["blocks"]), groups=int(st["groups"]),
                    mean_blocks_per_group=st["blocks"] / max(1, st["groups"]),
                    max_blocks_in_group=int(st["max_blocks_in_group"]),
                    finalized=int(st["finalized"]), state_peak_bytes=int(st["state_peak"]),
                    state_budget_bytes=int(state_budget or budget),
                    queued_peak=int(st["queued_peak"]),
                    median_rel_sigma_k_err_vs_known=float(np.median(errs)) if errs else None)

    sat = run(None)
    # each stream offers its bytes at a rate proportional to its size, so that all streams span
    # the same interval and the total offered load stays rho X throughout
    rng = np.random.default_rng(30001)
    arrivals = []
    for s_ in range(nstr):
        bytes_blk = 4.0 * draws.blocks[s_] * int(draws.n[s_])
        rate = args.serving_rho * sat["gbps"] * 1e9 * float(bytes_blk.sum()) / total_bytes
        gaps = rng.exponential(bytes_blk / rate)
        arrivals.append(np.cumsum(gaps))
    loaded = run(arrivals)
    # S2: a state budget of about 16 average footprints, and the stream requests themselves
    # arriving as a Poisson process at the rate that offers rho X in the long run; each stream's
    # blocks then arrive as a Poisson process at rho X / 16, so about 16 streams are open at a
    # time and admission (FIFO, by footprint) and continuous batching both engage
    rng2 = np.random.default_rng(30003)
    mean_bytes = total_bytes / nstr
    lam = args.serving_rho * sat["gbps"] * 1e9 / mean_bytes
    opens = np.cumsum(rng2.exponential(1.0 / lam, nstr))
    per_stream = args.serving_rho * sat["gbps"] * 1e9 / 16.0
    arr2 = []
    for s_ in range(nstr):
        bytes_blk = 4.0 * draws.blocks[s_] * int(draws.n[s_])
        arr2.append(opens[s_] + np.cumsum(rng2.exponential(bytes_blk / per_stream)))
    budget2 = int(16 * np.mean(foot))
    admission = run(arr2, state_budget=budget2, opens=opens)
    out = {"mode": mode, "streams": nstr, "data_gb": total_bytes / 1e9, "k": k, "l": l, "b": b,
           "saturated": sat, "rho": args.serving_rho, "poisson": loaded,
           "admission_s2": admission,
           "latency": "block submit (host) to the GPU completion of its grouped launch"}
    if host_too:
        # the same streams with their pools in pinned host memory: every block crosses PCIe into
        # one of 4 staging slots on the server's copy stream while earlier groups compute
        hpools = [p.cpu().pin_memory() for p in pools]
        pools.clear()
        torch.cuda.empty_cache()
        hsat = run(None, host=hpools)
        arr3 = []
        rng3 = np.random.default_rng(30005)
        for s_ in range(nstr):
            bytes_blk = 4.0 * draws.blocks[s_] * int(draws.n[s_])
            rate = args.serving_rho * hsat["gbps"] * 1e9 * float(bytes_blk.sum()) / total_bytes
            arr3.append(np.cumsum(rng3.exponential(bytes_blk / rate)))
        hload = run(arr3, host=hpools)
        hpools.clear()
        torch._C._host_emptyCache()
        out["host_pinned"] = {"staging_slots": 4, "saturated": hsat, "poisson": hload}
    pools.clear()
    return out


def h2d_peak(torch, gib=4):
    """Measured pinned host -> device copy rate (GB/s) of one large linear copy."""
    src = torch.empty(gib << 28, dtype=torch.float32, pin_memory=True)
    src.fill_(1.0)
    dst = torch.empty(gib << 28, dtype=torch.float32, device="cuda")
    best = 0.0
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        best = max(best, (gib << 30) / (time.perf_counter() - t0) / 1e9)
    del src, dst
    src_pools_release(torch)
    return best


def src_pools_release(torch):
    """Returns freed pinned host buffers to the system (torch caches them), so the next
    host-streamed workload can allocate its own."""
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    release = getattr(torch._C, "_host_emptyCache", None)
    if release is not None:
        release()
    return release is not None


def host_workload(args, torch, sk, which):
    """Host-streamed workloads: every row block is copied from pinned host memory by the library
    (side stream, staging ring of 3 slots) while the previous block is processed.

    host-c3: 1e6 x 1e4 FP32 (40 GB), Kronecker SVD (1000x1000 (x) 100x100) with
             sigma_j = |j^-2 + 1e-5 N(0,1)|, 8192-row blocks; modes FP32, BF16, BF16X2, FP8, all
             reading FP32 rows (the precision study: error against the known sigma).
    host-c5: 1.5e6 x 25000 FP32 (150 GB): 48 stacked copies of a 31250 x 25000 Kronecker SVD
             (125x250 (x) 125x200) scaled by 1/sqrt(48), so sigma(A) = |1/j + 1e-4 N(0,1)|
             exactly; 16384-row blocks sliced from a pinned pool (A0 plus 16384 rows); FP32 rows
             with FP32 compute against BF16 rows (the RNE of the pool) with BF16 compute."""
    import synth
    k, l, b = 50, 100, 10
    tmp = None
    peak = h2d_peak(torch, gib=1)
    print(f"[bench] pinned H2D peak {peak:.1f} GB/s", file=sys.stderr, flush=True)
    if which == "host-c3":
        m, n, blk, seed = 1_000_000, 10_000, 8192, 1003
        sig = synth.noisy_spectrum(synth.inv_square_spectrum(n), 1e-5, seed)
        K = synth.KronMatrix(1000, 1000, 100, 100, sig, seed)
        sigma = K.sigma
        print("[bench] generating 40 GB of pinned host rows", file=sys.stderr, flush=True)
        host = torch.empty(m, n, dtype=torch.float32, pin_memory=True)
        tmp = torch.empty(blk, n, dtype=torch.float32, device="cuda")
        for r0 in range(0, m, blk):
            c = min(blk, m - r0)
            K.rows_torch(r0, c, "cuda", out=tmp[:c])
            host[r0:r0 + c].copy_(tmp[:c])
        del tmp
        blocks = {"f32": [host[r0:r0 + blk] for r0 in range(0, m, blk)]}
        ref_blocks = [x.numpy() for x in blocks["f32"]]     # the reference reads the same rows
        ref_scale = 1.0
        modes = [("f32", "f32"), ("bf16", "f32"), ("bf16x2", "f32"), ("fp8", "f32")]
        desc = "host-streamed 1000000x10000 FP32 (40 GB pinned), k=50, l=100, b=10, 8192-row blocks"
    else:
        m0, copies, n, blk, seed = 31250, 48, 25000, 16384, 1005
        m = m0 * copies
        sig = synth.noisy_spectrum(synth.inv_spectrum(n), 1e-4, seed)
        P = synth.StackedPool(125, 250, 125, 200, copies, sig, seed, ext=blk)
        sigma = P.sigma
        print("[bench] generating the pinned pool (A0 + 16384 rows)", file=sys.stderr, flush=True)
        pool32 = torch.empty(P.m0 + P.ext, n, dtype=torch.float32, pin_memory=True)
        P.fill_pool(pool32, device="cuda")
        pool16 = torch.empty(P.m0 + P.ext, n, dtype=torch.bfloat16, pin_memory=True)
        pool16.copy_(pool32)
        blocks = {"f32": [], "bf16": []}
        for r0 in range(0, m, blk):
            a, e = P.slice_bounds(r0, min(blk, m - r0))
            blocks["f32"].append(pool32[a:e])
            blocks["bf16"].append(pool16[a:e])
        # Alg. 4 on A = [A0; ...; A0] (c copies) gives sqrt(c) times its result on A0: G is
        # [A0 Omega; ...], H = c A0^T A0 Omega, Q = (1 (x) Q0) / sqrt(c), B = sqrt(c) B0
        ref_blocks = [pool32[r0:min(r0 + blk, P.m0)].numpy() for r0 in range(0, P.m0, blk)]
        ref_scale = float(np.sqrt(copies))
        modes = [("bf16", "bf16"), ("f32", "f32")]
        desc = ("host-streamed 1500000x25000 FP32 (150 GB; 48 stacked 31250-row copies), k=50, "
                "l=100, b=10, 16384-row blocks")
    res = []
    for mode, src in modes:
        bl = blocks[src]
        es = 2 if src == "bf16" else 4
        h = sk.Sketch(n, m, blk, k, l, b, compute=mode, host_slots=3, host_src=src, seed=2000 + seed)
        for blkv in bl[:2]:                     # warmup: two blocks, then a fresh pass
            h.ingest(blkv)
        torch.cuda.synchronize()
        h.reset(2000 + seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for blkv in bl:
            h.ingest(blkv)
        torch.cuda.synchronize()
        t_pass = time.perf_counter() - t0
        S, V, _, rank = h.finalize(want_u=False)
        torch.cuda.synchronize()
        t_all = time.perf_counter() - t0
        Om = h.omega().cpu().numpy()
        h.close()
        S = S.cpu().numpy()
        wire = float(sum(int(x.shape[0]) for x in bl)) * n * es
        r = dict(dtype=mode, src=src, value=4.0 * m * n / t_all / 1e9, ms_per_step=t_all * 1e3,
                 pass_s=t_pass, finalize_s=t_all - t_pass, wire_gbps=wire / t_pass / 1e9,
                 pcie_frac=wire / t_pass / 1e9 / peak, rank=rank,
                 rel_sigma_k_err_vs_known=float(abs(S[k - 1] - sigma[k - 1]) / sigma[k - 1]),
                 max_rel_sigma_err_vs_known=float(np.max(np.abs(S - sigma[:k]) / sigma[:k])),
                 S=S, Om=Om)
        res.append(r)
        print(f"[bench] {mode}/{src}: {r['value']:.1f} GB/s FP32-eq, wire {r['wire_gbps']:.1f} GB/s",
              file=sys.stderr, flush=True)
    ref = res[[x["dtype"] for x in res].index("f32")]["S"]
    for r in res:
        r["max_rel_sigma_diff_vs_f32"] = float(np.max(np.abs(r["S"] - ref) / ref))
    cpu = None
    if args.check == "full":
        # FP64 reference with every mode's Omega' side by side (one pass over the rows; each
        # column group is an independent sketch), then the column-block loop and SVD per mode
        import oracle
        print("[bench] FP64 reference pass", file=sys.stderr, flush=True)
        Om_all = np.hstack([r["Om"] for r in res])
        t0 = time.perf_counter()
        G, H = oracle.sketch_pass((np.asarray(x, np.float64) for x in ref_blocks), Om_all)
        t_ref = time.perf_counter() - t0
        for i, r in enumerate(res):
            c = slice(i * l, (i + 1) * l)
            Q, Bm, _, _ = oracle.qb_from_sketch(G[:, c], H[:, c], r["Om"], b)
            Sr = oracle.svd_from_qb(Q, Bm, k, want_u=False)[0] * ref_scale
            e = np.abs(r["S"] - Sr) / Sr
            r["rel_sigma_k_err_vs_reference"] = float(e[k - 1])
            r["max_rel_sigma_err_vs_reference"] = float(e.max())
            r["gate_1e3"] = bool(e[k - 1] <= 1e-3)
        rows_ref = sum(x.shape[0] for x in ref_blocks)
        cpu = dict(value=4.0 * m * n / (t_ref * m / rows_ref / len(res)) / 1e9, unit="GB/s",
                   cores=host_cpu_info()[0], host_cores=host_cpu_info()[1], kind="oracle",
                   sample=f"FP64 reference pass over {rows_ref} rows with {len(res)} sketches of "
                          f"width {l} side by side ({t_ref:.1f} s), per sketch, scaled by "
                          f"m/{rows_ref}; finalize excluded")
    head = res[0]
    line = {
        "metric": METRIC, "value": head["value"], "unit": "GB/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head["dtype"], "data": "synthetic",
        "config": {"workload": desc, "m": m, "n": n, "k": k, "l": l, "b": b, "block_rows": blk,
                   "global_batch": m, "parallelism": "none"},
        "roofline": {"bound": "pcie", "achieved": head["wire_gbps"], "peak": peak, "unit": "GB/s",
                     "frac": head["pcie_frac"], "traffic": None,
                     "kernel": "host-to-device block copies (pinned, side stream)"},
        "cpu_baseline": cpu,
        "modes": [{kk: v for kk, v in r.items() if kk not in ("S", "Om")} for r in res],
    }
    # drop every reference to the pinned rows before handing them back
    blocks = ref_blocks = bl = blkv = host = pool32 = pool16 = None
    src_pools_release(torch)
    return line


def power_bench(mode, A, K, args, torch, sk):
    """The power scheme with P = 1 (Sec. 3.3, 4.2) on the resident workload: a first pass, Omega
    replaced by sqrt(n) orth(H), a second pass and the finalize (two reads of A).  Reports the
    time of the whole job, its FP32-equivalent rate per read of A, and the error against the
    known spectrum next to the single-pass error of the same mode."""
    m, n = A.shape
    sigma = K.sigma
    obj = sk.Sketch(n, m, args.block, args.k, args.l, args.b, compute=mode, seed=2002)

    def one_pass():
        for r0 in range(0, m, args.block):
            obj.ingest(A[r0:r0 + args.block])

    def job():
        obj.reset(2002)
        one_pass()
        route = obj.power_restart()
        one_pass()
        S, _, _, _ = obj.finalize(want_u=False)
        return S, route

    job()
    torch.cuda.synchronize()
    steps = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        S, route = job()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    S = S.cpu().numpy()
    obj.reset(2002)
    one_pass()
    S0, _, _, _ = obj.finalize(want_u=False)
    S0 = S0.cpu().numpy()
    obj.close()
    k = args.k
    rel1 = np.abs(S - sigma[:k]) / sigma[:k]
    rel0 = np.abs(S0 - sigma[:k]) / sigma[:k]
    print(f"[bench] power scheme {mode}: {ms:.2f} ms, rel sigma_k err vs known {rel1[-1]:.2e} "
          f"(single pass {rel0[-1]:.2e})", file=sys.stderr, flush=True)
    return {"dtype": mode, "passes": 2, "ms_per_job": ms,
            "value": 4.0 * m * n / (ms * 1e-3) / 1e9, "unit": "GB/s (FP32 A per job)",
            "per_read_gbps": 2 * 4.0 * m * n / (ms * 1e-3) / 1e9, "orth_route": route,
            "rel_sigma_k_err_vs_known": float(rel1[-1]),
            "max_rel_sigma_err_vs_known": float(rel1.max()),
            "single_pass_rel_sigma_k_err_vs_known": float(rel0[-1]),
            "single_pass_max_rel_sigma_err_vs_known": float(rel0.max())}


def accuracy_study(torch, sk):
    """Sec. 4.1's study: 3000 x 3000 matrices U diag(sigma) V^T (random orthogonal U, V) with the
    spectra Type 1-5, k = 50, l = 60, b = 10, in every compute mode, against the known spectrum
    (max |sigma_j - sigma_j(A)| over j <= k, the paper's max_err, and the relative error of
    sigma_k), the FP64 GPU result, the reference's Algorithm 4 and Algorithm 2 (same Omega)."""
    import oracle
    import synth
    N, k, l, b = 3000, 50, 60, 10
    print("[bench] accuracy study (Sec. 4.1): Types 1-5 x modes", file=sys.stderr, flush=True)
    rng = np.random.default_rng(4100)
    U = synth.orthonormal_factor(N, N, rng)
    V = synth.orthonormal_factor(N, N, rng)
    Om = synth.gaussian_omega(N, l, 4101)
    Omt = synth.gaussian_omega(N, l, 4102)
    out = []
    for kind in range(1, 6):
        s = synth.paper_type_spectrum(kind, N)
        A = (U * s) @ V.T
        row = {"type": kind}
        S64 = None
        for mode in ("f64", "f32", "bf16", "bf16x2", "fp8"):
            At = torch.from_numpy(A).to(torch.float64 if mode == "f64" else torch.float32).cuda()
            h = sk.Sketch(N, N, 1000, k, l, b, compute=mode, omega=Om)
            for r0 in range(0, N, 1000):
                h.ingest(At[r0:r0 + 1000])
            S, _, _, _ = h.finalize(want_u=False)
            torch.cuda.synchronize()
            h.close()
            S = S.cpu().numpy()
            if mode == "f64":
                S64 = S
            row[mode] = {"max_err": float(np.max(np.abs(S - s[:k]))),
                         "rel_sigma_k_err": float(abs(S[k - 1] - s[k - 1]) / s[k - 1]),
                         "max_rel_vs_f64": float(np.max(np.abs(S - S64) / S64))}
        r4 = oracle.single_pass_pca([A], Om, k, b, want_u=False)
        S2, _, _ = oracle.alg2_single_pass(A, Om, Omt, k, want_u=False)
        row["reference_alg4_max_err"] = float(np.max(np.abs(r4.S - s[:k])))
        row["reference_alg2_max_err"] = float(np.max(np.abs(S2 - s[:k])))
        out.append(row)
        print(f"[bench] Type {kind}: max_err f64 {row['f64']['max_err']:.2e} "
              f"f32 {row['f32']['max_err']:.2e} bf16 {row['bf16']['max_err']:.2e}; "
              f"reference Alg. 4 {row['reference_alg4_max_err']:.2e}, "
              f"Alg. 2 {row['reference_alg2_max_err']:.2e}", file=sys.stderr, flush=True)
    return {"workload": "3000x3000 U diag(sigma) V^T, Types 1-5, k=50, l=60, b=10, "
                        "1000-row device blocks", "rows": out}


def roofline(res, m, n, l, mode):
    """Dominant streaming kernel against its roof: HBM for the BF16/FP8 paths (algorithmic bytes
    = the block's FP32 bytes, read once per launch), the matrix-core peak for FP32/FP64
    (algorithmic flops = 2 l per element of the block, per launch)."""
    g2 = "k_gemm2" if mode == "f64" else "k_gemm2w + k_hsum"    # FP64 keeps the strip kernel
    dom, t = ("gemm1: g = a Omega (k_gemm1 + k_reduce1)", res["gemm1_ms"]) \
        if res["gemm1_ms"] >= res["gemm2_ms"] else \
        (f"gemm2: H += a^T g ({g2})", res["gemm2_ms"])
    if not t > 0:
        return None
    elems_per_launch = m * n / res["nblocks"]
    if mode in ("f32", "f64"):
        ach = 2.0 * l * elems_per_launch / (t * 1e-3) / 1e12
        peak = MFMA_PEAK_TFLOPS[mode]
        out = dict(bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak)
    else:
        ach = 4.0 * elems_per_launch / (t * 1e-3) / 1e9
        out = dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS)
    out["kernel"] = dom
    out["launch_us"] = t * 1e3
    out["traffic"] = traffic_for(dom.split(":")[0], mode)
    return out


def traffic_for(kernel, mode):
    """Counter-derived HBM bytes per launch of one product (its kernels summed) recorded in
    profiles/traffic.json, valid only while the kernel source is unchanged (its SHA-256 is stored
    next to the figure)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = os.path.join(ROOT, "paper_1704_07669_amd", "csrc", "pass.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
        ent = rec.get(f"{kernel}|{mode}")
        if ent and ent.get("pass_hip_sha256") == h:
            return ent["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def accuracy(A_host, K, res_modes, args):
    """Relative sigma errors of each mode against the FP64 reference on the stored A with the same
    Omega' (regenerated by the reference's own Philox/Box-Muller and rounding)."""
    import oracle
    m = A_host.shape[0]
    Om = oracle.gaussian_omega_philox(args.n, args.l, 2002)
    out = {}
    for res in res_modes:
        mode = res["mode"]
        Omq = oracle.quantize_omega(Om, mode)
        t0 = time.perf_counter()
        blocks = (A_host[r0:r0 + args.block] for r0 in range(0, m, args.block))
        ref = oracle.single_pass_pca(blocks, Omq, args.k, args.b, want_u=False)
        t_ref = time.perf_counter() - t0
        e = oracle.rel_sigma_error(res["S"], ref.S)
        out[mode] = dict(rel_sigma_k_err=float(e[args.k - 1]), max_rel_sigma_err=float(e.max()),
                         sin_theta_V=float(oracle.sin_theta_max(ref.V, res["V"])),
                         rel_sigma_k_err_vs_known=float(abs(res["S"][args.k - 1] - K.sigma[args.k - 1])
                                                        / K.sigma[args.k - 1]),
                         reference_seconds=t_ref, gate_1e3=bool(e[args.k - 1] <= 1e-3))
    return out


def host_cpu_info():
    """Threads the reference's BLAS runs with, and the host's logical / physical core counts."""
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 0) for d in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    return int(threads), dict(logical=os.cpu_count(), physical=phys)


def cpu_baseline(A_host, args):
    """The FP64 reference as it stands, timed on the host on a bounded sample: its pass
    (oracle.sketch_pass) over the leading row blocks until the time budget is spent, then its
    column-block loop and SVD (oracle.qb_from_sketch, oracle.svd_from_qb) on that sample's sketch;
    both are scaled linearly in m to the whole workload."""
    import oracle
    threads, host = host_cpu_info()
    m = A_host.shape[0]
    Om = oracle.gaussian_omega_philox(args.n, args.l, 2002)
    budget = args.cpu_seconds
    seen = [0]

    def sample_blocks(t_start):
        while seen[0] < m and time.perf_counter() - t_start < budget * 0.7:
            a = A_host[seen[0]:seen[0] + args.block]
            seen[0] += a.shape[0]
            yield a

    t0 = time.perf_counter()
    G, H = oracle.sketch_pass(sample_blocks(t0), Om)
    t_pass = time.perf_counter() - t0
    rows = seen[0]
    t1 = time.perf_counter()
    Q, B, _, _ = oracle.qb_from_sketch(G, H, Om, args.b)
    oracle.svd_from_qb(Q, B, args.k, want_u=False)
    t_fin = time.perf_counter() - t1
    scale = m / rows
    t_est = (t_pass + t_fin) * scale
    return dict(value=4.0 * m * args.n / t_est / 1e9, unit="GB/s", cores=threads, kind="oracle",
                host_cores=host,
                sample=f"oracle.sketch_pass over the first {rows} of {m} rows ({rows // args.block}"
                       f" blocks, {t_pass:.1f} s) plus qb_from_sketch and svd_from_qb on that "
                       f"sketch ({t_fin:.1f} s), scaled by m/{rows}")


def main():
    args = parse()
    if args.b <= 0:
        args.b = args.l
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1704_07669_amd as sk
    sk.load_library()
    torch.cuda.set_device(0)
    if args.workload != "fp32-resident":
        print(json.dumps(host_workload(args, torch, sk, args.workload)))
        return
    print(f"[bench] generating A {args.m}x{args.n} FP32 on the GPU", file=sys.stderr, flush=True)
    A, K = make_matrix(args, torch)
    modes = [args.mode] + [c for c in args.compare.split(",")
                           if c and c != "none" and c != args.mode]
    results = []
    for mode in modes:
        print(f"[bench] mode {mode}: {args.warmup} warmup + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        results.append(bench_mode(mode, A, args, torch, sk))
        print(f"[bench] mode {mode}: {results[-1]['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    power = [power_bench(mode, A, K, args, torch, sk) for mode in args.power.split(",") if mode]
    p50, p99 = block_latency(A, args, torch, sk, args.mode)
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 1073741824 bytes read, 1073741824 bytes written",
              file=sys.stderr, flush=True)
        del src, dst
    head = results[0]
    acc, cpu = {}, None
    serving = []
    if args.serving_streams > 0:
        A_keep = A
        for smode in [x for x in args.serving_modes.split(",") if x]:
            print(f"[bench] serving scenario, {args.serving_streams} streams, {smode}",
                  file=sys.stderr, flush=True)
            serving.append(serving_bench(args, torch, sk, smode,
                                         host_too=bool(args.serving_host) and not serving))
            print(f"[bench] serving {smode}: saturated {serving[-1]['saturated']['gbps']:.1f} GB/s,"
                  f" p99 {serving[-1]['poisson']['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
            if "host_pinned" in serving[-1]:
                hp = serving[-1]["host_pinned"]
                print(f"[bench] serving {smode} from pinned host: saturated "
                      f"{hp['saturated']['gbps']:.1f} GB/s, p99 {hp['poisson']['p99_ms']:.2f} ms",
                      file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        A = A_keep
    if args.check == "full" or args.cpu_seconds > 0:
        print("[bench] copying A to the host for the reference", file=sys.stderr, flush=True)
        A_host = A.cpu().numpy()
        del A
        torch.cuda.empty_cache()
        if args.check == "full":
            print("[bench] FP64 reference accuracy check", file=sys.stderr, flush=True)
            acc = accuracy(A_host, K, results, args)
        if args.cpu_seconds > 0:
            print("[bench] CPU baseline (reference on a bounded sample)", file=sys.stderr,
                  flush=True)
            cpu = cpu_baseline(A_host, args)
        del A_host
    study = accuracy_study(torch, sk) if args.study else None
    configs = []
    for w in [x for x in args.host_configs.split(",") if x]:
        print(f"[bench] host-streamed workload {w}", file=sys.stderr, flush=True)
        configs.append(host_workload(args, torch, sk, "host-" + w))
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["mode"],
        "data": "synthetic",
        "config": {"workload": f"fp32-resident {args.m}x{args.n}, k={args.k}, l={args.l}, "
                               f"b={args.b}, {args.block}-row blocks",
                   "m": args.m, "n": args.n, "k": args.k, "l": args.l, "b": args.b,
                   "block_rows": args.block, "global_batch": args.m, "parallelism": "none"},
        "roofline": roofline(head, args.m, args.n, args.l, head["mode"]),
        "cpu_baseline": cpu,
        "per_step_ms": {"g = a Omega": head["gemm1_ms"] * head["nblocks"],
                        "H += a^T g": head["gemm2_ms"] * head["nblocks"],
                        "finalize": head["finalize_ms"]},
        "pass_only_gbps": 4.0 * args.m * args.n / ((head["gemm1_ms"] + head["gemm2_ms"]) *
                                                   head["nblocks"] * 1e-3) / 1e9,
        "block_latency_ms": {"p50": p50, "p99": p99, "rows": args.block},
        "serving": serving,
        "accuracy": acc.get(head["mode"]),
        "compare": [
            {"dtype": r["mode"], "value": r["value"], "ms_per_step": r["ms_per_step"],
             "roofline": roofline(r, args.m, args.n, args.l, r["mode"]),
             "per_step_ms": {"g = a Omega": r["gemm1_ms"] * r["nblocks"],
                             "H += a^T g": r["gemm2_ms"] * r["nblocks"],
                             "finalize": r["finalize_ms"]},
             "accuracy": acc.get(r["mode"])} for r in results[1:]],
        "power_scheme": power,
        "accuracy_study": study,
        "configs": configs,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
