"""Benchmark of the sparse-coding hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 6,000,000
synthetic SH rest vectors (d = 45), each an exact 4-sparse combination of a
K = 512 Gaussian unit-norm dictionary (coefficients U[-1,1]) plus N(0, sigma=1e-3)
noise; k = 12, eps = 1e-2.  The support proposer is trained first (untimed)
on 2,000,000 signals of the same generator labelled by the FP32 encoder.

One step = the whole hot path over the batch: the learned+BF16 encoder (BF16
MFMA proposer -> top-24 candidates -> restricted Batch-OMP -> full-OMP
fallback, whose correlations D^T x run on BF16 matrix cores as six split-BF16
products of FP32 accuracy, on the signals whose residual exceeds eps), then
the radiance of every code at one view direction per Gaussian.  Inputs are
resident in HBM before timing.  The comparators (plain FP32 Batch-OMP, the
BF16 precision form alone, the learned encoder with an FP32-correlation
fallback, an untrained proposer, correlation screening) are timed on the
same inputs and reported beside it, and so is the 16-scene batch (sizes
log-uniform in 50k..6M, K in {128, 256, 512}, k in {4, 8, 12, 16}, eps = 0)
encoded in one autotuned persistent launch and as one launch per scene.

Prints ONE JSON line.  `python bench.py --gpus N` with N > 1 exits: the
encoder is measured on one GPU.
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_errors(D, X, k, eps, gpu, sample, threads):
    """Codes of the seeded subsample `sample` against the FP64 oracle's:
    aggregate residual gap (negative = below the oracle's greedy path), the
    99th percentile and maximum of |r_gpu - r_oracle| / ||x|| per signal,
    and the share of signals with another support."""
    import oracle
    ref = oracle.omp(D, X[sample], k, eps, nthreads=threads)
    gi, gr = gpu[0], gpu[3].astype(np.float64)
    rr = ref["resid"]
    xn = np.linalg.norm(X[sample].astype(np.float64), axis=1)
    agg = np.sqrt((rr ** 2).sum())
    dev = np.abs(gr - rr) / np.maximum(xn, 1e-30)
    return {"sample": int(len(sample)), "resid_gap": float((np.sqrt((gr ** 2).sum()) - agg) / agg),
            "resid_dev_p99": float(np.quantile(dev, 0.99)), "resid_dev_max": float(dev.max()),
            "support_mismatch": float(np.mean(np.any(gi != ref["idx"], axis=1)))}


def other_workloads(args, log, sc, I, autotune, torch, dev, stream, ev):
    """The SH-like and precision-form workloads, each timed as a step on its
    own (inputs resident), with roofline fractions and errors against the FP64
    oracle on a seeded subsample."""
    threads = len(os.sched_getaffinity(0))
    rng = np.random.Generator(np.random.PCG64(12))
    out = {}

    def time_steps(fn, nmarks):
        for _ in range(args.warmup):
            fn([ev() for _ in range(nmarks)])
        torch.cuda.synchronize()
        rec = []
        for _ in range(args.steps):
            m = [ev() for _ in range(nmarks)]
            fn(m)
            rec.append(m)
        torch.cuda.synchronize()
        return [float(np.mean([m[i].elapsed_time(m[i + 1]) for m in rec])) for i in range(nmarks - 1)]

    # SH-like coefficients, K = 256 dictionary learned by MOD, k = 8, eps = 1e-3, one view per Gaussian
    t0 = time.perf_counter()
    w = I.workload_sh_like(N=1_000_000)
    D2 = np.load(os.path.join(ROOT, "tests", "golden", "sh_like_dict_K256.npy"))
    X2 = torch.from_numpy(w["X"]).to(dev)
    dir2 = torch.from_numpy(w["dirs"]).to(dev)
    N2, k2, e2 = X2.shape[0], w["k"], w["eps"]
    h2 = sc.gram_precompute(torch.from_numpy(D2).to(dev))
    tune2 = autotune.tune_dictionary(h2, X2, k2, e2, use_cache=False)
    o2 = sc.omp_encode(h2, X2, k2, e2)
    rgb2 = torch.empty((N2, 3), dtype=torch.float32, device=dev)

    def step2(m):
        m[0].record(stream)
        sc.omp_encode(h2, X2, k2, e2, out=o2)
        m[1].record(stream)
        sc.sh_eval_sparse(h2, o2[0], o2[1], o2[2], dir2, sc.DIRS_PER_SIGNAL, out=rgb2)
        m[2].record(stream)
    sc.omp_stats(h2, reset=True)
    ph = time_steps(step2, 3)
    st = sc.omp_stats(h2)
    cnt = o2[2].cpu().numpy()
    codes = [t.cpu().numpy() for t in o2]
    sample = np.sort(rng.choice(N2, min(args.oracle_sample, N2), replace=False))
    err = oracle_errors(D2, w["X"], k2, e2, [c[sample] for c in codes], sample, threads)
    fl = batch_omp_flops(D2.shape[0], 45, cnt)
    nnz = float(np.maximum(cnt, 0).sum())
    rad_bytes = 8.0 * nnz + 28.0 * N2
    out["sh_like_K256_k8"] = {
        "workload": "1e6 SH-like rest vectors (Laplace 0.3*2^-l per band, RGB rho=0.8), K=256 MOD dictionary, "
                    "k=8, eps=1e-3, FP32; step = encode + one-view radiance",
        "N": N2, "ms_per_step": round(ph[0] + ph[1], 4), "ms_encode": round(ph[0], 4), "ms_radiance": round(ph[1], 4),
        "gaussians_per_s": round(N2 / ((ph[0] + ph[1]) * 1e-3), 1), "mean_atoms": round(nnz / N2, 4),
        "encode_roofline": {"bound": "alu", "achieved": round(fl / (ph[0] * 1e-3) / 1e12, 3),
                            "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": round(fl / (ph[0] * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4)},
        "radiance_roofline": {"bound": "hbm", "achieved": round(rad_bytes / (ph[1] * 1e-3) / 1e9, 1),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(rad_bytes / (ph[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              "bytes_per_gaussian": "8 per non-zero + 28"},
        "fp64_refit_rate": st["fp64_refits"] / (N2 * (args.steps + args.warmup)),
        "vs_oracle": err, "encoder_tuning": tune2}
    log(f"SH-like workload {ph} ms, error {err} ({time.perf_counter() - t0:.1f} s)")
    h2.destroy()
    del X2, dir2, o2, rgb2

    # precision form: K = 512, k = 12, eps = 0, 5% near-duplicate signals; FP32 and split-BF16 correlations
    t0 = time.perf_counter()
    w = I.workload_precision(N=3_000_000)
    D3 = w["D"]
    X3 = torch.from_numpy(w["X"]).to(dev)
    N3, k3 = X3.shape[0], w["k"]
    h3 = sc.gram_precompute(torch.from_numpy(D3).to(dev))
    tune3 = autotune.tune_dictionary(h3, X3, k3, 0.0, use_cache=False)
    tune3["row_cache_bf16"] = autotune.tune_dictionary(h3, X3, k3, 0.0, sc.PREC_BF16, use_cache=False)["row_cache_bf16"]
    o3 = sc.omp_encode(h3, X3, k3, 0.0)
    sample = np.sort(rng.choice(N3, min(args.oracle_sample, N3), replace=False))
    rows = {}
    for name, flags in (("fp32", 0), ("bf16_precision_form", sc.PREC_BF16)):
        def step3(m, flags=flags):
            m[0].record(stream)
            sc.omp_encode(h3, X3, k3, 0.0, flags, out=o3)
            m[1].record(stream)
        sc.omp_stats(h3, reset=True)
        ph = time_steps(step3, 2)
        st = sc.omp_stats(h3)
        codes = [t.cpu().numpy() for t in o3]
        cnt = codes[2]
        fl = batch_omp_flops(D3.shape[0], 45, cnt)
        rows[name] = {"ms": round(ph[0], 4), "gaussians_per_s": round(N3 / (ph[0] * 1e-3), 1),
                      "roofline": {"bound": "alu", "achieved": round(fl / (ph[0] * 1e-3) / 1e12, 3),
                                   "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(fl / (ph[0] * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4)},
                      "fp64_refit_rate": st["fp64_refits"] / (N3 * (args.steps + args.warmup)),
                      "vs_oracle": oracle_errors(D3, w["X"], k3, 0.0, [c[sample] for c in codes], sample, threads)}
        log(f"precision workload {name}: {ph[0]:.2f} ms, {rows[name]['vs_oracle']}")
    out["precision_K512_k12_neardup"] = {
        "workload": "3e6 signals, 4-sparse over a K=512 Gaussian unit-norm dictionary + N(0,sigma=1e-3) noise, "
                    "5% near-duplicate rows (copies + N(0,1e-4^2)), k=12, eps=0",
        "N": N3, "encoder_tuning": tune3, **rows}
    log(f"precision workload done in {time.perf_counter() - t0:.1f} s")
    h3.destroy()
    del X3, o3
    torch.cuda.empty_cache()
    return out


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
    ap.add_argument("--no-batched", action="store_true", help="skip the 16-scene batched comparator")
    ap.add_argument("--no-sweep", action="store_true", help="skip the tolerance / CSC storage sweep")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the SH-like (1M, K=256) and precision-form (3M, K=512) workload lines")
    ap.add_argument("--oracle-sample", type=int, default=200_000,
                    help="seeded subsample of those workloads checked against the FP64 oracle")
    ap.add_argument("--proposer-weights", default=None,
                    help="FP32 parameter file (.npy): loaded instead of training when it exists, else written "
                         "after training (lets counter passes reuse the proposer a traced run trained)")
    ap.add_argument("--tuning", default=None,
                    help="JSON file of the encoder and restricted-cap tuning: applied when it exists, else written "
                         "after tuning")
    ap.add_argument("--quick", action="store_true",
                    help="headline step only, then a 1 GiB device copy (profiling and counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the encoder shards by rows with no exchange, "
              "and this encoder is measured on a single GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2605_30396_amd import autotune
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

    # ---- CPU baseline: the FP64 oracle on a bounded sample (run before the GPU
    # work; its codes also serve as the reference for the error columns) ----
    cpu, cpu_ref = None, None
    if not args.no_cpu_baseline:
        import oracle
        ns = min(args.cpu_sample, N)
        threads = len(os.sched_getaffinity(0))
        tc = time.perf_counter()
        cpu_ref = oracle.omp(D, X[:ns], k, eps, nthreads=threads)
        dtc = time.perf_counter() - tc
        cpu = {"value": round(ns / dtc, 1), "unit": "Gaussians/s", "cores": threads, "kind": "oracle",
               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "sample": f"first {ns} of the {N} signals, FP64 OMP (Householder-QR least squares), "
                         f"{threads} threads, {dtc:.1f} s"}
        log(f"CPU oracle baseline: {cpu['value']:.0f} Gaussians/s on {threads} threads")

    # a saved tuning (--tuning) is applied instead of searching, so a profiled
    # run launches the step's kernels in the timed configuration only
    saved = None
    if args.tuning and os.path.exists(args.tuning):
        with open(args.tuning) as f:
            saved = json.load(f)

    # ---- autotune the FP32 encoder on a slice (untimed) ----
    if saved:
        tuned = saved["encoder"]
        h.set_tuning(sc.TUNE_FP32_CORRELATION, tuned["corr"])
        h.set_tuning(sc.TUNE_ROW_CACHE, tuned["row_cache"])
        if "row_cache_bf16" in tuned:
            h.set_tuning(sc.TUNE_ROW_CACHE_BF16, tuned["row_cache_bf16"])
    else:
        tuned = autotune.tune_dictionary(h, Xg, k, eps, use_cache=False)
        tuned["row_cache_bf16"] = autotune.tune_dictionary(h, Xg, k, eps, sc.PREC_BF16,
                                                           use_cache=False)["row_cache_bf16"]
    log(f"encoder tuning {tuned}")

    # ---- train the proposer (untimed) ----
    t1 = time.perf_counter()
    prop = sc.proposer_create(d, 256, K)
    prop.set_params(I.mlp_init(I.rng_for(5), d, 256, K))
    if args.proposer_weights and os.path.exists(args.proposer_weights):
        prop.set_params(torch.from_numpy(np.load(args.proposer_weights, allow_pickle=False)))
        hist = {"loss": [float("nan")]}
        log(f"proposer weights loaded from {args.proposer_weights}")
    else:
        sup, cnt = trainer.omp_labels(h, Xtr_g, k, eps)
        hist = trainer.train(prop, Xtr_g, sup, cnt, epochs=args.epochs, batch=1024, lr=3e-3, pos_weight=8.0, seed=1)
        hist["recall_train"] = trainer.support_recall(prop, Xtr_g[:20000], sup[:20000], cnt[:20000])
        del sup, cnt
        if args.proposer_weights:
            np.save(args.proposer_weights, prop.get_params().cpu().numpy())
    train_s = time.perf_counter() - t1
    log(f"proposer ready in {train_s:.1f} s, loss {hist['loss'][-1]:.4f}")
    del Xtr_g
    untrained = sc.proposer_create(d, 256, K)
    untrained.set_params(I.mlp_init(I.rng_for(5), d, 256, K))
    # restricted-step cap of the learned encoder (untimed)
    if saved:
        tuned_learned = saved["learned"]
        h.set_tuning(sc.TUNE_RESTRICTED_CAP, tuned_learned["restricted_cap"])
    else:
        tuned_learned = autotune.tune_learned(h, prop, Xg, k, eps, sc.PREC_BF16, use_cache=False)
        if args.tuning:
            with open(args.tuning, "w") as f:
                json.dump({"encoder": tuned, "learned": tuned_learned}, f)
    log(f"learned tuning {tuned_learned}")

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
        """The learned encoder as its three stages (events between them);
        p = None: correlation screening in place of the network."""
        marks[0].record(stream)
        if p is None:
            sc.screen_topk(h, Xg, N_CAND, cand=cand)
        else:
            sc.proposer_forward(p, Xg, N_CAND, cand=cand)
        marks[1].record(stream)
        sc.omp_encode_restricted(h, Xg, k, eps, cand, flags & ~sc.PREC_BF16, out=out, miss_rows=miss_rows,
                                 miss_count=miss_count)
        marks[2].record(stream)
        sc.omp_encode_rows(h, Xg, miss_rows, miss_count, N, k, eps, out, flags)
        marks[3].record(stream)

    def time_variant(run, nmarks, steps=None, warmup=None):
        steps = args.steps if steps is None else steps
        for _ in range(args.warmup if warmup is None else warmup):
            run([ev() for _ in range(nmarks)])
        torch.cuda.synchronize()
        sc.omp_stats(h, reset=True)
        rec = []
        tw = time.perf_counter()
        for _ in range(steps):
            m = [ev() for _ in range(nmarks)]
            run(m)
            rec.append(m)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - tw) / steps
        st = sc.omp_stats(h)
        phases = [float(np.mean([m[i].elapsed_time(m[i + 1]) for m in rec])) for i in range(nmarks - 1)]
        return wall * 1e3, phases, st

    qs = np.random.Generator(np.random.PCG64(11)).choice(len(cpu_ref["resid"]) if cpu_ref else N, 4000,
                                                          replace=False)
    qsg = torch.from_numpy(qs).to(dev)

    def quality():
        """Mean atoms per code and, when the CPU baseline ran, the error of
        the codes in the output buffers against its FP64 codes on 4000 sampled
        signals: aggregate residual gap (negative = lower residual than the
        oracle's greedy path), share of signals whose residual exceeds the
        oracle's by more than 1e-3 relative, share with another support."""
        cnt = count.float()
        q = {"mean_atoms": round(float(cnt[cnt >= 0].mean().item()), 4)}
        if cpu_ref is None:
            return q
        rg = resid[qsg].cpu().numpy().astype(np.float64)
        gi = idx[qsg].cpu().numpy()
        rr = cpu_ref["resid"][qs]
        agg_r = np.sqrt((rr ** 2).sum())
        q.update(resid_gap=float((np.sqrt((rg ** 2).sum()) - agg_r) / agg_r),
                 worse_than_oracle=float(np.mean(rg > rr * (1 + 1e-3) + 1e-7)),
                 support_mismatch=float(np.mean(np.any(gi != cpu_ref["idx"][qs], axis=1))))
        return q

    results = {}

    # ---- headline: learned+BF16 encoder + radiance, one step ----
    def headline(marks):
        learned_step(prop, sc.PREC_BF16, marks)
        sc.sh_eval_sparse(h, idx, coef, count, dirg, sc.DIRS_PER_SIGNAL, out=rgb)
        marks[4].record(stream)

    head_ms_step, ph, st = time_variant(headline, 5)
    results["learned_bf16"] = dict(ms=sum(ph[:3]), phases_ms=dict(proposer=ph[0], restricted=ph[1], fallback=ph[2]),
                                   fallback_frac=st["fallbacks"] / (N * args.steps), **quality())
    eval_ms = ph[3]
    # the same codes' radiance from CSC columns (packed untimed): reads only the non-zeros
    colptr_h, rows_h, vals_h = sc.pack_csc(idx, coef, count)
    def csc_eval(m):
        m[0].record(stream)
        sc.sh_eval_csc(h, colptr_h, rows_h, vals_h, dirg, sc.DIRS_PER_SIGNAL, out=rgb)
        m[1].record(stream)
    _, ph_csc, _ = time_variant(csc_eval, 2)
    nnz_head = int(colptr_h[-1].item())
    csc_radiance = {"ms": round(ph_csc[0], 4), "nnz": nnz_head,
                    "bytes": 8 * nnz_head + 32 * N,
                    "achieved": round((8 * nnz_head + 32 * N) / (ph_csc[0] * 1e-3) / 1e9, 1), "unit": "GB/s",
                    "peak": HBM_PEAK_GBS,
                    "frac": round((8 * nnz_head + 32 * N) / (ph_csc[0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "bytes_per_gaussian": "8 per non-zero (index + value) + 8 column pointer + 12 direction + "
                                          "12 rgb"}
    del colptr_h, rows_h, vals_h
    fb_rows = int(miss_count.item())
    cnt_head = count.cpu().numpy()
    miss_np = miss_rows[:fb_rows].cpu().numpy()
    log(f"headline step {head_ms_step:.2f} ms, phases {ph}")
    if args.quick:
        # a plain device copy of known size, for scaling the HBM counters
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"quick": True, "ms_per_step": head_ms_step, "phases_ms": ph, "N": N,
                          "fallback_rows": fb_rows, "copy_bytes": 1 << 30}))
        return

    for name, flags in (("plain_fp32", 0), ("bf16_precision_form", sc.PREC_BF16)):
        def run(m, flags=flags):
            m[0].record(stream)
            sc.omp_encode(h, Xg, k, eps, flags, out=out)
            m[1].record(stream)
        _, ph2, st2 = time_variant(run, 2)
        results[name] = dict(ms=ph2[0], **quality())
        log(f"{name} {ph2[0]:.2f} ms")
    _, ph2, st2 = time_variant(lambda m: learned_step(prop, 0, m), 4)
    results["learned_bf16_proposer_fp32_fallback"] = dict(ms=sum(ph2), phases_ms=dict(proposer=ph2[0],
                                                                                     restricted=ph2[1],
                                                                                     fallback=ph2[2]),
                                                          fallback_frac=st2["fallbacks"] / (N * args.steps),
                                                          **quality())
    _, ph2, st2 = time_variant(lambda m: learned_step(untrained, sc.PREC_BF16, m), 4)
    results["learned_untrained"] = dict(ms=sum(ph2), phases_ms=dict(proposer=ph2[0], restricted=ph2[1],
                                                                   fallback=ph2[2]),
                                        fallback_frac=st2["fallbacks"] / (N * args.steps), **quality())
    _, ph2, st2 = time_variant(lambda m: learned_step(None, sc.PREC_BF16, m), 4)
    results["screened_top24"] = dict(ms=sum(ph2), phases_ms=dict(screen=ph2[0], restricted=ph2[1],
                                                                fallback=ph2[2]),
                                     fallback_frac=st2["fallbacks"] / (N * args.steps), **quality())
    lab = trainer.omp_labels(h, Xg[:20000], k, eps)
    recall = trainer.support_recall(prop, Xg[:20000], *lab)
    recall0 = trainer.support_recall(untrained, Xg[:20000], *lab)
    scr = sc.screen_topk(h, Xg[:20000], N_CAND).cpu().numpy()
    li, lc = (t.cpu().numpy() for t in lab)
    recall_screen = float(np.mean([set(li[i, :max(lc[i], 0)]) <= set(scr[i]) for i in range(len(scr))]))
    for v in results.values():
        v["gaussians_per_s"] = round(N / (v["ms"] * 1e-3), 1)

    # ---- the other single-GPU workloads: SH-like (1M, K=256, k=8) and the
    # precision form (3M, K=512, k=12, eps=0, 5% near-duplicates) ----
    workloads = None
    if not args.no_workloads:
        del cand, miss_rows
        torch.cuda.empty_cache()
        workloads = other_workloads(args, log, sc, I, autotune, torch, dev, stream, ev)

    # ---- the 16-scene batch in one persistent launch ----
    batched = None
    if not args.no_batched:
        del rgb, dirg
        torch.cuda.empty_cache()
        tb = time.perf_counter()
        specs = I.scene_batch_specs()
        scenes, hs = [], []
        for sp in specs:
            Ds, Xs = I.scene_inputs(sp)
            hq = sc.gram_precompute(torch.from_numpy(Ds).to(dev))
            hs.append(hq)
            scenes.append(dict(dict=hq, X=torch.from_numpy(Xs).to(dev), k=sp["k"], eps=0.0))
            del Xs
        Nb = sum(sp["N"] for sp in specs)
        log(f"batched inputs ({Nb} signals) in {time.perf_counter() - tb:.1f} s")
        tuning, tms = autotune.tune_batched(scenes, sample=1 << 18, use_cache=False)
        outs = sc.omp_encode_batched(scenes, tuning)
        for _ in range(args.warmup):
            sc.omp_encode_batched(scenes, tuning)
        torch.cuda.synchronize()
        tms_list = []
        for _ in range(args.steps):
            a, b = ev(), ev()
            a.record(stream)
            outs = sc.omp_encode_batched(scenes, tuning)
            b.record(stream)
            tms_list.append((a, b))
        torch.cuda.synchronize()
        bms = float(np.mean([a.elapsed_time(b) for a, b in tms_list]))
        bflops = 0.0
        for q, sp in enumerate(specs):
            bflops += batch_omp_flops(sp["K"], d, outs[q][2].cpu().numpy())
        # the same scenes as one launch per scene, each with its own tuned encoder
        per_out = []
        for sc_ in scenes:
            autotune.tune_dictionary(sc_["dict"], sc_["X"], sc_["k"], 0.0, use_cache=False)
            Ns = sc_["X"].shape[0]
            per_out.append((torch.empty((Ns, sc_["k"]), dtype=torch.int32, device=dev),
                            torch.empty((Ns, sc_["k"]), dtype=torch.float32, device=dev),
                            torch.empty((Ns,), dtype=torch.int32, device=dev),
                            torch.empty((Ns,), dtype=torch.float32, device=dev)))

        def per_scene():
            for sc_, o in zip(scenes, per_out):
                sc.omp_encode(sc_["dict"], sc_["X"], sc_["k"], 0.0, out=o)
        for _ in range(args.warmup):
            per_scene()
        torch.cuda.synchronize()
        tps = []
        for _ in range(args.steps):
            a, b = ev(), ev()
            a.record(stream)
            per_scene()
            b.record(stream)
            tps.append((a, b))
        torch.cuda.synchronize()
        pms = float(np.mean([a.elapsed_time(b) for a, b in tps]))
        batched = dict(workload="16 scenes, N log-uniform 50k..6M (seed 4), K in {128,256,512}, "
                                "k in {4,8,12,16}, eps=0, one persistent launch",
                       N=Nb, ms=round(bms, 3), gaussians_per_s=round(Nb / (bms * 1e-3), 1),
                       tuning=tuning.as_dict(), tflops=round(bflops / (bms * 1e-3) / 1e12, 3),
                       per_scene_launches_ms=round(pms, 3))
        log(f"batched {bms:.2f} ms for {Nb} signals, tuning {tuning.as_dict()}; per-scene launches {pms:.2f} ms")
        del per_out
        for hq in hs:
            hq.destroy()
        del scenes, outs

    # ---- tolerance sweep with CSC storage on SH-like coefficients ----
    sweep = None
    if not args.no_sweep:
        from paper_2605_30396_amd import storage
        t_s = time.perf_counter()
        w2 = I.workload_sh_like(N=1_000_000)
        D2 = np.load(os.path.join(ROOT, "tests", "golden", "sh_like_dict_K256.npy"))
        X2 = torch.from_numpy(w2["X"]).to(dev)
        N2, K2, k2 = X2.shape[0], D2.shape[0], 32
        h2 = sc.gram_precompute(torch.from_numpy(D2).to(dev))
        autotune.tune_dictionary(h2, X2, k2, 0.1, sc.EPS_RELATIVE, use_cache=False)
        rng2 = np.random.default_rng(57)
        pos2 = torch.from_numpy(rng2.normal(scale=3.0, size=(N2, 3)).astype(np.float32)).to(dev)
        dc2 = torch.from_numpy(rng2.normal(scale=1.0, size=(N2, 3)).astype(np.float32)).to(dev)
        x2n = float(torch.linalg.vector_norm(X2.double()).item())
        sweep = {"workload": "1e6 SH-like rest vectors (Laplace 0.3*2^-l per band, RGB rho=0.8), K=256 MOD "
                             "dictionary, relative tolerance, k=32", "points": []}

        def evt(fn):
            a, b = ev(), ev()
            fn()
            torch.cuda.synchronize()
            a.record(stream)
            r = fn()
            b.record(stream)
            torch.cuda.synchronize()
            return a.elapsed_time(b), r
        for tol in (0.03, 0.05, 0.1, 0.2):
            t_enc, codes = evt(lambda: sc.omp_encode(h2, X2, k2, tol, sc.EPS_RELATIVE))
            i2, c2, n2, r2 = codes
            t_pack, packed = evt(lambda: sc.pack_csc(i2, c2, n2))
            colptr2, rows2, vals2 = packed
            t_col, _ = evt(lambda: sc.gaussian_rgb_csc(h2, colptr2, rows2, vals2, pos2, dc2, (0.0, 0.0, 10.0)))
            nnz = int(colptr2[-1].item())
            sweep["points"].append({
                "tol": tol, "ms_encode": round(t_enc, 3), "ms_pack_csc": round(t_pack, 3),
                "ms_colour_step": round(t_col, 4), "mean_atoms": round(nnz / N2, 3),
                "compression_ratio": round(storage.compression_ratio(N2, nnz, K2), 3),
                "rel_sh_error": round(float(torch.linalg.vector_norm(r2.double()).item()) / x2n, 5)})
        # the dictionary half of one learning pass (MOD from the tol = 0.1 codes), and the encoder
        # writing CSC directly at that tolerance
        i2, c2, n2, r2 = sc.omp_encode(h2, X2, k2, 0.1, sc.EPS_RELATIVE)
        t_mod, (_, nrep) = evt(lambda: sc.mod_update(X2, i2, c2, n2, r2, K2))
        t_csc, _ = evt(lambda: sc.omp_encode_csc(h2, X2, k2, 0.1, sc.EPS_RELATIVE))
        sweep["mod_update"] = {"ms": round(t_mod, 3), "atoms_replaced": int(nrep), "N": N2, "K": K2,
                               "codes": "tol 0.1, k 32"}
        sweep["encode_csc_one_pass_tol0.1_ms"] = round(t_csc, 3)
        log(f"tolerance sweep in {time.perf_counter() - t_s:.1f} s: {sweep['points']}, MOD {t_mod:.2f} ms, "
            f"encode to CSC {t_csc:.2f} ms")
        h2.destroy()
        del X2, pos2, dc2

    # ---- per-kernel rates of the headline step, roofline of the dominant one ----
    phs = results["learned_bf16"]["phases_ms"]
    ok = np.ones(N, bool)
    ok[miss_np] = False
    n_ok = cnt_head[ok].astype(np.float64)
    kern = {
        "proposer": dict(kernel="proposer_topk_kernel", bound="mfma", unit="TFLOP/s", peak=BF16_MFMA_PEAK_TFLOPS,
                         achieved=MLP_FLOPS * N / (phs["proposer"] * 1e-3) / 1e12,
                         src=("proposer.hip", "mfma.h", "wave.h", "sc_internal.h")),
        "restricted": dict(kernel="omp_restricted_kernel", bound="alu", unit="TFLOP/s", peak=FP32_VALU_PEAK_TFLOPS,
                           achieved=float(np.sum(2.0 * N_CAND * d + N_CAND * n_ok * (n_ok + 1))) /
                           (phs["restricted"] * 1e-3) / 1e12, src=("romp.hip", "wave.h", "sc_internal.h")),
        "fallback": dict(kernel="omp_batch_kernel", bound="alu", unit="TFLOP/s", peak=FP32_VALU_PEAK_TFLOPS,
                         achieved=batch_omp_flops(K, d, cnt_head[miss_np]) / (phs["fallback"] * 1e-3) / 1e12,
                         src=("omp_core.h", "omp_batch_impl.h", "omp_batch_bf16.hip", "omp_batch_mfma.hip",
                              "omp_batch_valu.hip", "mfma.h", "wave.h", "sc_internal.h")),
        "radiance": dict(kernel="sh_eval_kernel", bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                         achieved=sh_eval_bytes(N, k) / (eval_ms * 1e-3) / 1e9, src=("sh_eval.hip", "sh_basis.h", "sc_internal.h")),
        "radiance_nonzero_bytes": dict(kernel="sh_eval_kernel", bound="hbm", unit="GB/s", peak=HBM_PEAK_GBS,
                                       achieved=(8 * float(np.maximum(cnt_head, 0).sum()) + 28 * N) /
                                       (eval_ms * 1e-3) / 1e9, src=("sh_eval.hip", "sh_basis.h", "sc_internal.h")),
    }
    for v in kern.values():
        v["frac"] = round(v["achieved"] / v["peak"], 4)
        v["achieved"] = round(v["achieved"], 3)
    dom = max(("proposer", "restricted", "fallback"), key=lambda q: phs[q])
    kd = kern[dom]
    roof = {"bound": kd["bound"], "kernel": kd["kernel"], "achieved": kd["achieved"], "peak": kd["peak"],
            "unit": kd["unit"], "frac": kd["frac"],
            "traffic": read_traffic(kd["kernel"], kernel_source_hash(*kd["src"]))}
    per_kernel = {q: {kk: v[kk] for kk in ("kernel", "bound", "achieved", "peak", "unit", "frac")} | {
        "ms": round(phs[q] if q in phs else eval_ms, 4)} for q, v in kern.items()}
    per_kernel["radiance_nonzero_bytes"]["note"] = ("the padded-code kernel's rate counted against the method's "
                                                    "own bytes, 8 per non-zero + 28 per Gaussian")

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
                               "U[-1,1] + N(0,sigma=1e-3) noise, k=12, eps=1e-2, top-24 candidates; step = learned+BF16 "
                               "encode (BF16 proposer, split-BF16 correlations in the full-OMP fallback) + one-view "
                               "radiance",
                   "N": N, "K": K, "k": k, "eps": eps, "n_cand": N_CAND, "encoder_tuning": tuned,
                   "learned_tuning": tuned_learned},
        "speedup_vs_plain_fp32": (round(plain["ms"] / results["learned_bf16"]["ms"], 4) if plain else None),
        "comparators": {k2: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                        for k2, v in results.items()},
        "workloads": workloads,
        "batched": batched,
        "tolerance_sweep": sweep,
        "radiance_from_csc": csc_radiance,
        "kernels": per_kernel,
        "training": {"seconds": round(train_s, 2), "epochs": args.epochs, "train_N": args.train_N,
                     "final_loss": round(hist["loss"][-1], 5), "recall_at_24": recall,
                     "recall_at_24_train": hist.get("recall_train"),
                     "recall_at_24_untrained": recall0, "recall_at_24_screening": recall_screen},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out_json))
    prop.destroy()
    untrained.destroy()
    h.destroy()


if __name__ == "__main__":
    main()
