"""Benchmark of the sparse-coding hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 6,000,000
synthetic SH rest vectors (d = 45), each an exact 4-sparse combination of a
K = 512 Gaussian unit-norm dictionary (coefficients U[-1,1]) plus N(0, sigma=1e-3)
noise; k = 12, eps = 1e-2.  The support proposer is trained first (untimed)
on 2,000,000 signals of the same generator labelled by the FP32 encoder.

One step = the whole hot path over the batch: the learned encoder (BF16 MFMA
proposer -> top-24 candidates -> restricted Batch-OMP -> full-OMP fallback on
the signals whose residual exceeds eps), then the radiance of every code at
one view direction per Gaussian.  Inputs are resident in HBM before timing.
The comparators (plain FP32 Batch-OMP, BF16 precision form, untrained
proposer) are timed on the same inputs and reported beside it.

Prints ONE JSON line.  `python bench.py --gpus N` with N > 1 exits: this
build runs on one GPU.
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

METRIC = "Gaussians sparse-coded/s at K=512,k=12: learned+BF16 vs plain FP32, same error"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3     # published vector FP32 (packed FMA); 78.6 without packed FMA
BF16_MFMA_PEAK_TFLOPS = 2500.0
MLP_FLOPS = 2 * (45 * 256 + 256 * 256 + 256 * 512)   # 416,256 per signal
N_CAND = 24


def batch_omp_flops(K, d, counts):
    """Algorithmic FLOPs of Batch-OMP: alpha0 = D^T x (2Kd) plus, at step n,
    the correlation update with the n selected Gram columns (2Kn)."""
    n = np.asarray(counts, np.float64)
    n = n[n >= 0]
    return float(np.sum(2.0 * K * d + K * n * (n + 1)))


def sh_eval_bytes(N, k):
    """HBM bytes of the radiance kernel per Gaussian and view: codes 8k (int32
    index + float32 coefficient), count 4, direction 12, rgb 12."""
    return N * (8 * k + 28)


def kernel_source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2605_30396_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel, src_hash):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE
    (profiles/traffic_<kernel>.txt), if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != src_hash:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=6_000_000)
    ap.add_argument("--train-N", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=6_000_000)
    ap.add_argument("--quick", action="store_true", help="headline step only (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the encoder shards by rows with no exchange, "
              "and multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2605_30396_amd import inputs as I
    from paper_2605_30396_amd import sc, trainer

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    K, k, eps, d = 512, 12, 1e-2, 45
    t0 = time.perf_counter()
    D = I.learned_dictionary(K)
    X = I.learned_eval_signals(D, N=args.N)
    Xtr = I.learned_train_signals(D, N=args.train_N)
    N = X.shape[0]
    dirs = I.unit_directions(I.rng_for(56), N)
    log(f"inputs generated in {time.perf_counter() - t0:.1f} s")
    Xg, Xtr_g = torch.from_numpy(X).to(dev), torch.from_numpy(Xtr).to(dev)
    dirg = torch.from_numpy(dirs).to(dev)
    h = sc.gram_precompute(torch.from_numpy(D).to(dev))

    # ---- autotune the FP32 correlation stage on a slice (untimed) ----
    sl = Xg[:262144]
    best = None
    for corr in (sc.CORR_VALU, sc.CORR_MFMA):
        h.set_tuning(sc.TUNE_FP32_CORRELATION, corr)
        sc.omp_encode(h, sl, k, eps)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sc.omp_encode(h, sl, k, eps)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        if best is None or ms < best[1]:
            best = (corr, ms)
    h.set_tuning(sc.TUNE_FP32_CORRELATION, best[0])

    # ---- train the proposer (untimed) ----
    t1 = time.perf_counter()
    sup, cnt = trainer.omp_labels(h, Xtr_g, k, eps)
    prop = sc.proposer_create(d, 256, K)
    prop.set_params(I.mlp_init(I.rng_for(5), d, 256, K))
    hist = trainer.train(prop, Xtr_g, sup, cnt, epochs=args.epochs, batch=1024, lr=3e-3, pos_weight=8.0, seed=1)
    train_s = time.perf_counter() - t1
    log(f"proposer trained in {train_s:.1f} s, loss {hist['loss'][-1]:.4f}")
    untrained = sc.proposer_create(d, 256, K)
    untrained.set_params(I.mlp_init(I.rng_for(5), d, 256, K))

    # ---- buffers ----
    idx = torch.empty((N, k), dtype=torch.int32, device=dev)
    coef = torch.empty((N, k), dtype=torch.float32, device=dev)
    count = torch.empty((N,), dtype=torch.int32, device=dev)
    resid = torch.empty((N,), dtype=torch.float32, device=dev)
    out = (idx, coef, count, resid)
    rgb = torch.empty((N, 3), dtype=torch.float32, device=dev)
    cand = torch.empty((N, N_CAND), dtype=torch.int32, device=dev)
    miss_rows = torch.empty((N,), dtype=torch.int32, device=dev)
    miss_count = torch.zeros((1,), dtype=torch.int32, device=dev)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def learned_step(p, flags, marks):
        """The learned encoder as its three kernels (events between them)."""
        marks[0].record(stream)
        sc.proposer_forward(p, Xg, N_CAND, cand=cand)
        marks[1].record(stream)
        sc.omp_encode_restricted(h, Xg, k, eps, cand, flags & ~sc.PREC_BF16, out=out, miss_rows=miss_rows,
                                 miss_count=miss_count)
        marks[2].record(stream)
        sc.omp_encode_rows(h, Xg, miss_rows, miss_count, N, k, eps, out, flags)
        marks[3].record(stream)

    def time_variant(run, nmarks):
        for _ in range(args.warmup):
            run([ev() for _ in range(nmarks)])
        torch.cuda.synchronize()
        sc.omp_stats(h, reset=True)
        rec = []
        tw = time.perf_counter()
        for _ in range(args.steps):
            m = [ev() for _ in range(nmarks)]
            run(m)
            rec.append(m)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - tw) / args.steps
        st = sc.omp_stats(h)
        phases = [float(np.mean([m[i].elapsed_time(m[i + 1]) for m in rec])) for i in range(nmarks - 1)]
        return wall * 1e3, phases, st

    qs = np.random.Generator(np.random.PCG64(11)).choice(N, 4000, replace=False)
    qref = {}

    def quality():
        """Error of the codes in the output buffers against the FP64 oracle on
        4000 sampled signals: aggregate residual gap (negative = lower residual
        than the oracle's greedy path), share of signals whose residual exceeds
        the oracle's by more than 1e-3 relative, share with another support."""
        import oracle
        if not qref:
            qref.update(oracle.omp(D, X[qs], k, eps))
        rg = resid[torch.from_numpy(qs).to(dev)].cpu().numpy().astype(np.float64)
        gi = idx[torch.from_numpy(qs).to(dev)].cpu().numpy()
        rr = qref["resid"]
        agg_r = np.sqrt((rr ** 2).sum())
        return dict(resid_gap=float((np.sqrt((rg ** 2).sum()) - agg_r) / agg_r),
                    worse_than_oracle=float(np.mean(rg > rr * (1 + 1e-3) + 1e-7)),
                    support_mismatch=float(np.mean(np.any(gi != qref["idx"], axis=1))))

    results = {}
    cnt_np = {}
    # headline: learned (BF16 proposer) + radiance, as one step
    def headline(marks, p=prop, flags=0):
        learned_step(p, flags, marks)
        sc.sh_eval_sparse(h, idx, coef, count, dirg, sc.DIRS_PER_SIGNAL, out=rgb)
        marks[4].record(stream)

    ms_step, ph, st = time_variant(headline, 5)
    results["learned_bf16_proposer"] = dict(ms=sum(ph[:3]), phases_ms=dict(proposer=ph[0], restricted=ph[1],
                                                                          fallback=ph[2]),
                                            fallback_frac=st["fallbacks"] / (N * args.steps), **quality())
    eval_ms = ph[3]
    head_ms_step = ms_step
    fb_rows = int(miss_count.item())
    cnt_head = count.cpu().numpy()
    miss_np = miss_rows[:fb_rows].cpu().numpy()
    if not args.quick:
        for name, flags in (("plain_fp32", 0), ("bf16_precision_form", sc.PREC_BF16)):
            def run(m, flags=flags):
                m[0].record(stream)
                sc.omp_encode(h, Xg, k, eps, flags, out=out)
                m[1].record(stream)
            ms, ph2, st2 = time_variant(run, 2)
            results[name] = dict(ms=ph2[0], **quality())
            cnt_np[name] = count.cpu().numpy()
        ms, ph2, st2 = time_variant(lambda m: learned_step(prop, sc.PREC_BF16, m), 4)
        results["learned_bf16_fallback"] = dict(ms=sum(ph2), phases_ms=dict(proposer=ph2[0], restricted=ph2[1],
                                                                           fallback=ph2[2]),
                                                fallback_frac=st2["fallbacks"] / (N * args.steps), **quality())
        ms, ph2, st2 = time_variant(lambda m: learned_step(untrained, 0, m), 4)
        results["learned_untrained"] = dict(ms=sum(ph2), phases_ms=dict(proposer=ph2[0], restricted=ph2[1],
                                                                       fallback=ph2[2]),
                                            fallback_frac=st2["fallbacks"] / (N * args.steps), **quality())
        recall = trainer.support_recall(prop, Xg[:20000], *trainer.omp_labels(h, Xg[:20000], k, eps))
    else:
        recall = None
    for v in results.values():
        v["gaussians_per_s"] = round(N / (v["ms"] * 1e-3), 1)

    # ---- roofline of the dominant kernel of the headline step ----
    phs = results["learned_bf16_proposer"]["phases_ms"]
    dom = max(phs, key=phs.get)
    if dom == "proposer":
        ach = MLP_FLOPS * N / (phs[dom] * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "proposer_topk_kernel<4>", "achieved": round(ach, 3),
                "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s"}
        tk = "proposer_topk_kernel"
        src = kernel_source_hash("proposer.hip", "mfma.h")
    elif dom == "fallback":
        fl = batch_omp_flops(K, d, cnt_head[miss_np])
        ach = fl / (phs[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "omp_batch_kernel<8,12> (fallback rows)", "achieved": round(ach, 3),
                "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s"}
        tk = "omp_batch_kernel"
        src = kernel_source_hash("omp_batch.hip")
    else:
        ok = np.ones(N, bool)
        ok[miss_np] = False
        n = cnt_head[ok].astype(np.float64)
        fl = float(np.sum(2.0 * N_CAND * d + N_CAND * n * (n + 1)))
        ach = fl / (phs[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": "omp_restricted_kernel<12>", "achieved": round(ach, 3),
                "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s"}
        tk = "omp_restricted_kernel"
        src = kernel_source_hash("romp.hip")
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = read_traffic(tk, src)

    # ---- CPU baseline: the FP64 oracle on a bounded sample ----
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns = min(args.cpu_sample, N)
        threads = len(os.sched_getaffinity(0))
        tc = time.perf_counter()
        oracle.omp(D, X[:ns], k, eps, nthreads=threads)
        dtc = time.perf_counter() - tc
        cpu = {"value": round(ns / dtc, 1), "unit": "Gaussians/s", "cores": threads, "kind": "oracle",
               "sample": f"first {ns} of the {N} signals, FP64 OMP (Householder-QR least squares), "
                         f"{threads} threads, {dtc:.1f} s"}

    plain = results.get("plain_fp32")
    out_json = {
        "metric": METRIC,
        "value": round(N / (head_ms_step * 1e-3), 1),
        "unit": "Gaussians/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head_ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32",
        "data": "synthetic",
        "config": {"workload": "learned-form: N=6e6 signals d=45, K=512 Gaussian unit-norm dictionary, 4-sparse "
                               "U[-1,1] + N(0,sigma=1e-3) noise, k=12, eps=1e-2, top-24 candidates; step = learned encode "
                               "+ one-view radiance",
                   "N": N, "K": K, "k": k, "eps": eps, "n_cand": N_CAND,
                   "fp32_correlation": "mfma" if best[0] == sc.CORR_MFMA else "valu"},
        "speedup_vs_plain_fp32": (round(plain["ms"] / results["learned_bf16_proposer"]["ms"], 4) if plain else None),
        "comparators": {k2: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k2, v in results.items()},
        "radiance": {"ms": round(eval_ms, 4), "GB_per_s": round(sh_eval_bytes(N, k) / (eval_ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(sh_eval_bytes(N, k) / (eval_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "training": {"seconds": round(train_s, 2), "epochs": args.epochs, "train_N": args.train_N,
                     "final_loss": round(hist["loss"][-1], 5), "recall_at_24": recall},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out_json))
    prop.destroy()
    untrained.destroy()
    h.destroy()


if __name__ == "__main__":
    main()
