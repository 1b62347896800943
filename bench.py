"""Benchmark: strike grids per second, batched SFFT vs dense FFT at n = 24.

Workload: 4096 seeded Heston instances drawn over the batched parameter box
(kappa~U[0.5,4], theta~U[0.01,0.1], sigma_v~U[0.1,0.8], rho~U[-0.9,-0.1], v0~U[0.01,0.1],
T~U[0.1,2]), S0=100, r=0.03, alpha=1.5, Simpson weights, n forced to 24,
eta = 40/2^12; complex64 contraction with FP64 factorisation, tolerance 1e-8.
One step = the whole SFFT chain for the batch: QTT construction, SFFT apply (zip-up),
TT rounding and readout of 4096 near-money prices per instance (the Q_n operator is built
once and cached), replayed as one captured HIP graph. A strike grid = one instance's priced
M-point log-strike grid: the rounded output train, from which every grid price is readable,
plus its 4096 read-out prices. Per-stage times come from HIP events on eager steps.
The dense Stockham path (all 2^24 prices per instance written to HBM) is timed on the
same problems for comparison, and the same draws with uneven n ~ U{16..28} (slot counts
autotuned, longest chain first) give the ragged-batch figure.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import cm_workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_TFLOPS = 78.6
FP32_VECTOR_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--n", type=int, default=24)
    ap.add_argument("--dense-instances", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-vg", action="store_true")
    ap.add_argument("--no-qft", action="store_true")
    ap.add_argument("--no-mpo-table", action="store_true")
    ap.add_argument("--slots", type=int, nargs=3, metavar=("BUILD", "APPLY", "ROUND"), default=[4096, 1536, 4096],
                    help="persistent-workgroup counts of the three sweep ops (default: what autotune_slots picks "
                         "for this workload on MI355X, and the counts the committed profiles were taken with)")
    ap.add_argument("--autotune", action="store_true", help="time the candidate slot counts first and use the best")
    ap.add_argument("--default-slots", action="store_true", help="library default slot counts (min(batch, 2048))")
    ap.add_argument("--shots", type=int, default=4096, help="measurement shots per instance in the QFT-observable "
                    "section (the paper's hardware default)")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager steps instead of graph replays "
                    "(for counter-collection runs)")
    ap.add_argument("--copy-calibration", action="store_true", help="run one 1 GiB device copy first: the "
                    "reference a traffic counter is scaled by")
    ap.add_argument("--surrogate-steps", type=int, default=60000)
    ap.add_argument("--curves", action="store_true", help="instead of the benchmark line, print one JSON "
                    "line per n of the paper's memory / rank / time / NRMSE curves (Section 4)")
    ap.add_argument("--curves-n", type=int, nargs=2, default=(3, 40))
    ap.add_argument("--curves-dense-max", type=int, default=30)
    ap.add_argument("--curves-tol", type=float, default=1e-10, help="SFFT (zip-up and rounding) tolerance of the curves")
    ap.add_argument("--curves-mpo-tol", type=float, default=None, help="operator rounding tolerance of the curves "
                    "(default: a tenth of --curves-tol)")
    ap.add_argument("--curves-list", type=int, nargs="*", default=None, help="explicit grid exponents instead of "
                    "the --curves-n range")
    ap.add_argument("--curves-shots", type=int, default=4096)
    ap.add_argument("--sweep", action="store_true", help="instead of the benchmark line, print one JSON line per "
                    "grid exponent of --sweep-list: the batched SFFT chain and the dense complex64 FFT on the same "
                    "seeded Heston draws with n fixed (grids/s of each)")
    ap.add_argument("--sweep-list", type=int, nargs="*", default=[12, 14, 16, 18, 20, 22, 24, 26, 28])
    ap.add_argument("--curves-build-tol", type=float, default=None, help="QTT construction tolerance of the curves "
                    "(default: a tenth of --curves-tol)")
    return ap.parse_args()


def zipup_flops(xr, wr, yr_zip, n):
    """Algorithmic FP operations of one zip-up (per instance), from the bond dimensions:
    (FP32 flops, FP64 flops). Per site: the complex64 contraction
    chi*w*2*r*r' + chi*2*w*2*w'*r' complex MACs (8 real flops each); the FP64 pivoted
    Householder QR of the (2chi) x (w'r') matrix stopped at rank k,
    sum_{i<k} 16 (m-i)(p-i) (reflector application) plus 8 (m-i)(p-i) (norm refresh);
    and forming Q_k, sum_{i<k} 16 (m-i) k."""
    f32 = f64 = 0.0
    chi = 1
    for l in range(n):
        w0, w1, r0, r1 = wr[l], wr[l + 1], xr[l], xr[l + 1]
        f32 += 8.0 * (chi * w0 * 2 * r0 * r1 + chi * 2 * w0 * 2 * w1 * r1)
        if l < n - 1:
            m, p = 2 * chi, w1 * r1
            k = yr_zip[l + 1]
            for i in range(k):
                f64 += 24.0 * (m - i) * (p - i) + 16.0 * (m - i) * k
            chi = k
    return f32, f64


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def round_flops(yz, yr, n, d=2):
    """FP64 flops of cm_tt_round on a zip-up output (left-orthonormal, so the first sweep is
    skipped), from its bonds before (yz) and after (yr) rounding. Right to left, bond
    l = n-1 .. 1: the core l (yz_l x d x yz_{l+1}) times the carry (yz_{l+1} x yr_{l+1}),
    8 yz_l d yz_{l+1} yr_{l+1}; the pivoted Householder QR of its conjugate transpose
    (d yr_{l+1} rows, yz_l columns) to the kept rank k = yr_l, sum_{i<k} 24 (m-i)(p-i) as in
    zipup_flops; one one-sided Jacobi sweep over the k x k factor (the three inner products
    of every column pair, the least any Jacobi SVD does), 12 k^2 (k-1); then core 0,
    8 d yz_1 yr_1."""
    f = 0.0
    for l in range(n - 1, 0, -1):
        kl, kr, rpp, k = int(yz[l]), int(yz[l + 1]), int(yr[l + 1]), int(yr[l])
        f += 8.0 * kl * d * kr * rpp
        m, pcols = d * rpp, kl
        for i in range(min(k, m, pcols)):
            f += 24.0 * (m - i) * (pcols - i)
        f += 12.0 * k * k * (k - 1)
    f += 8.0 * d * int(yz[1]) * int(yr[1])
    return f


def readout_flops(yr, n, strikes):
    """FP32 flops of the read-out with shared suffixes, the least a right-to-left
    contraction of the output train needs for this strike set: the partial contraction of
    cores l..n-1 depends on u >> l only, so level l costs one vector-matrix product
    (8 r_l r_{l+1} flops) per distinct u >> l."""
    u = np.asarray(strikes, dtype=np.int64)
    return float(sum(len(np.unique(u >> l)) * 8.0 * int(yr[l]) * int(yr[l + 1]) for l in range(n)))


def core_elems(rk, n, d=2):
    """Complex elements of a train's cores at bonds rk."""
    return int(sum(int(rk[l]) * d * int(rk[l + 1]) for l in range(n)))


# The per-grid operation counts the scope table quotes for the SFFT at n = 24 (chi ~ 9,
# w ~ 10, r ~ 7): zip-up contraction 6.5e6 complex64 flops, zip-up factorisations 1.6e7
# FP64 flops, rounding 1e6, read-out 5e6 (FP32), construction 3e6 (FP64).
SURVEY_ZIPUP_F32, SURVEY_ZIPUP_F64, SURVEY_ROUND_F64, SURVEY_READ_F32, SURVEY_BUILD_F64 = 6.5e6, 1.6e7, 1e6, 5e6, 3e6


def alu_roofline(kernel, ms, f32, f64, algo_bytes, traffic_name=None, sources=None, extra=None):
    """Fraction of the mixed FP32/FP64 vector roof, sum_i flops_i / peak_i over the time,
    with the achieved FP64-equivalent rate, the algorithmic HBM bytes and (when counters
    for the current sources exist) the measured traffic and its ratio to them."""
    t = ms * 1e-3
    frac = (f32 / (FP32_VECTOR_TFLOPS * 1e12) + f64 / (FP64_VECTOR_TFLOPS * 1e12)) / t
    rec = {"kernel": kernel, "bound": "alu", "achieved": frac * FP64_VECTOR_TFLOPS, "peak": FP64_VECTOR_TFLOPS,
           "unit": "TFLOP/s (FP64-equivalent: FP32 flops count 78.6/157.3)", "frac": frac, "ms": ms,
           "flops_fp32": f32, "flops_fp64": f64, "algorithmic_bytes": algo_bytes,
           "hbm_frac_of_algorithmic_bytes": algo_bytes / t / (HBM_PEAK_GBS * 1e9)}
    if traffic_name:
        tr = profiled_traffic(traffic_name, sources)
        rec["traffic"] = tr
        rec["traffic_per"] = PROFILED_TRAFFIC[traffic_name]["per"]
        rec["traffic_over_algorithmic"] = (tr / algo_bytes) if tr else None
    if extra:
        rec.update(extra)
    return rec


def cpu_baseline(problems, timed: int = 3):
    """The oracle's dense pricing (psi on all 2^n points, FFT, readout) timed on the host:
    one untimed warm-up grid (instance 0), then `timed` further grids (instances 1..timed)
    each timed on its own; the value is one over the median time. numpy's FFT and
    elementwise kernels run on one thread, and any BLAS pool is held to one thread as well,
    so the figure is per core. Returns the timing record and the oracle's prices of every
    grid priced, which the price-error figures of the GPU paths are checked against."""
    from oracle import carr_madan as O
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:   # pragma: no cover
        threadpool_limits = None
    priced, times = [], []
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        priced.append((0, O.prices_dense(problems[0])))
        for b in range(1, 1 + min(timed, len(problems) - 1)):
            t0 = time.perf_counter()
            priced.append((b, O.prices_dense(problems[b])))
            times.append(time.perf_counter() - t0)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    med = float(np.median(times))
    n = problems[0].n
    rec = {"value": 1.0 / med, "unit": "strike grids/s", "cores": 1, "kind": "oracle",
           "sample": f"{len(times)} dense Heston grids at n={n} (instances 1..{len(times)} of the workload, after one "
                     f"untimed warm-up grid) priced by the numpy FP64 oracle (psi on all 2^{n} points + FFT + readout) "
                     f"on one thread; median {med:.2f} s per grid (times {', '.join(f'{t:.2f}' for t in times)} s)",
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    return rec, priced


def oracle_errors(samples):
    """Part of the cpu_baseline leg: the largest |GPU - oracle| / S0 over sampled
    (problem, strike indices, GPU prices) triples, the oracle's direct sums running on
    host threads over the samples."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import carr_madan as O

    def one(smp):
        p, u, got = smp
        return float(np.abs(got - O.prices_direct(p, u)).max() / p.S0)

    with ThreadPoolExecutor(8) as ex:
        errs = list(ex.map(one, samples))
    return max(errs), errs


def parity_sample(probs, got, strikes, idx, every: int = 16):
    """(problem, every `every`-th read-out strike, its GPU price) for instances idx: what the
    cpu_baseline leg checks against the oracle."""
    return [(probs[b], strikes[b][::every].copy(), got[b][::every].copy()) for b in idx]


def ragged_run(cm, torch, batch, nk, steps, parity=True):
    """The same parameter draws with n ~ U{16..28}: slot counts autotuned per sweep op,
    longest chain first, whole chain captured as one HIP graph. The price error is taken
    against the oracle on eight instances (the first two at n = 28 and six spread over the
    batch), at every 16th read-out strike."""
    probs = W.heston_batch(batch, seed=20261203, n_range=(16, 28))
    ns = sorted(set(p.n for p in probs))
    strikes = torch.from_numpy(np.stack([W.near_money(p, nk) for p in probs])).cuda()
    mpo = cm.MpoCache(ns, 1e-9, 32, cm.CM_C64)
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32, mpo=mpo)
    slots = cm.autotune_slots(pr, strikes, candidates=SLOT_CANDIDATES, reps=1)
    pr.capture(strikes)
    pr.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pr.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = pr.statuses()
    out = {"grids_per_s": batch / dt, "ms_per_step": dt * 1e3, "slots": slots,
           "status_errors": {k: int((v != 0).sum()) for k, v in st.items()},
           "n_hist": {int(n): sum(1 for p in probs if p.n == n) for n in ns}}
    if parity:
        at28 = [b for b, p in enumerate(probs) if p.n == 28][:2]
        idx = at28 + [b for b in range(0, batch, max(1, batch // 6)) if b not in at28][:6]
        out["_parity"] = parity_sample(probs, pr.graph_prices.cpu().numpy(), strikes.cpu().numpy(), idx)
        out["err_sample"] = (f"{len(idx)} instances (n = {', '.join(str(probs[b].n) for b in idx)}) x {nk // 16} "
                             f"strikes against the oracle's direct sums")
    return out


def vg_run(cm, torch, batch, nk, steps, n, parity=True):
    """Variance Gamma (the model named with the gamma time change in Section 2): seeded
    draws over a box of equity-index-like fits, the same SFFT chain at the same n, graph
    replay; the price error against the oracle's direct sums on four of the instances, at
    every 16th read-out strike."""
    probs = W.vg_batch(batch, seed=31, n=n)
    strikes = torch.from_numpy(np.stack([W.near_money(p, nk) for p in probs])).cuda()
    mpo = cm.MpoCache([n], 1e-9, 32, cm.CM_C64)
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32, mpo=mpo)
    pr.capture(strikes)
    pr.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pr.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = pr.statuses()
    out = {"grids_per_s": batch / dt, "ms_per_step": dt * 1e3,
           "status_errors": {k: int((v != 0).sum()) for k, v in st.items()},
           "y_max_rank": int(pr.y.ranks[:, : n + 1].max().item())}
    if parity:
        idx = list(range(0, batch, max(1, batch // 4)))[:4]
        out["_parity"] = parity_sample(probs, pr.graph_prices.cpu().numpy(), strikes.cpu().numpy(), idx)
        out["err_sample"] = f"{len(idx)} instances x {nk // 16} strikes against the oracle's direct sums"
    return out


# persistent-workgroup counts tried by the autotuner: multiples of the 256 CUs up to one
# workgroup per instance
SLOT_CANDIDATES = (768, 1024, 1536, 2048, 3072, 4096)


def mpo_table_run(cm, torch, n_lo=1, n_hi=40, tol=1e-9, cap=32, reps=3):
    """The operator look-up table: Q_n for every n in [n_lo, n_hi] (complex64, the bench
    chain's operator tolerance) built by one cm_qft_mpo_table launch, against one
    cm_qft_mpo call per n, and against loading the saved table from a file."""
    import tempfile

    def best(fn):
        t = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
        return t

    box = {}
    t_table = best(lambda: box.__setitem__("m", cm.MpoCache(range(n_lo, n_hi + 1), tol, cap, cm.CM_C64)))
    m = box["m"]
    single = cm.TTBatch([n if n >= n_lo else 0 for n in range(n_hi + 1)], 2, 2, cap, cm.CM_C64)
    ws = cm.Workspace()

    def seq():
        for n in range(n_lo, n_hi + 1):
            cm.cm_qft_mpo(n, tol, cap, single, n, ws)

    t_seq = best(seq)
    identical = bool(torch.equal(single.cores, m.w.cores) and torch.equal(single.ranks, m.w.ranks))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "qft_table.npz")
        m.save(path)
        size = os.path.getsize(path)
        t_load = best(lambda: cm.MpoCache.load(path))
    return {"n_range": [n_lo, n_hi], "tol": tol, "cap": cap, "table_build_ms": t_table * 1e3,
            "one_call_per_n_ms": t_seq * 1e3, "load_from_file_ms": t_load * 1e3, "file_bytes": size,
            "max_rank": int(m.w.rank_max), "table_equals_per_n_builds": identical}


def sampler_flops(rk, n, shots, ones):
    """Algorithmic FP64 flops of the sampler on one train: at level t every shot forms
    w0 = w Y_t[:,0,:] (8 r_t r_{t+1}) and its mass w0 E w0^H from the upper triangle
    (4 r(r-1) + 8 r with r = r_{t+1}); shots whose bit t is 1 repeat both for bit 1."""
    f = 0.0
    for t in range(n):
        ra, rb = int(rk[t]), int(rk[t + 1])
        per = 8 * ra * rb + 4 * rb * (rb - 1) + 8 * rb
        f += per * (shots + int(ones[t]))
    return f


def qft_run(cm, torch, pr, strikes, shots, steps):
    """The QFT-observable arm (Section 2.2) emulated on the output trains of the main
    workload: `shots` measurement outcomes per instance (uniforms drawn on the device
    from a seeded generator), outcome counts at the read-out strikes and the observable
    prices from them, next to the exact-probability observable read-out. The error of the
    shot prices against the exact observable prices is the estimator's shot noise."""
    batch, n = pr.batch, int(pr.y.struct.n_max)
    dev = "cuda"
    stream = torch.cuda.current_stream()
    g = torch.Generator(device=dev)
    g.manual_seed(4242)
    U = torch.rand((batch, n, shots), dtype=torch.float64, device=dev, generator=g)
    samples = torch.empty((batch, shots), dtype=torch.int64, device=dev)
    norm2 = torch.empty(batch, dtype=torch.float64, device=dev)
    st = torch.zeros(batch, dtype=torch.int32, device=dev)
    st_shot = torch.zeros(batch, dtype=torch.int32, device=dev)
    nk = strikes.shape[-1]
    counts = torch.empty((batch, nk), dtype=torch.int32, device=dev)
    shot_px = torch.empty((batch, nk), dtype=torch.float64, device=dev)
    exact_px = torch.empty((batch, nk), dtype=torch.float64, device=dev)
    ws = cm.Workspace(dev)

    def once(ev=None):
        if ev:
            ev[0].record(stream)
        cm.cm_sample_outcomes(pr.y, U, shots, samples, norm2, st, ws)
        if ev:
            ev[1].record(stream)
        cm.cm_shot_prices(pr.prob, batch, norm2, samples, shots, strikes, nk, counts, shot_px, st_shot)
        if ev:
            ev[2].record(stream)
        cm.cm_readout_observable(pr.y, pr.prob, strikes, nk, exact_px, st_shot)
        if ev:
            ev[3].record(stream)

    once()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    acc = [0.0, 0.0, 0.0]
    for _ in range(steps):
        once(ev)
        torch.cuda.synchronize()
        for i in range(3):
            acc[i] += ev[i].elapsed_time(ev[i + 1])
    sample_ms, shot_ms, exact_ms = (a / steps for a in acc)
    sm = samples.cpu().numpy()
    rk = pr.y.ranks.cpu().numpy()
    flops = 0.0
    for b in range(batch):
        nb = pr.ns[b]
        ones = ((sm[b][:, None] >> np.arange(nb)) & 1).sum(axis=0)
        flops += sampler_flops(rk[b], nb, shots, ones)
    achieved = flops / (sample_ms * 1e-3) / 1e12
    sp, ep = shot_px.cpu().numpy(), exact_px.cpu().numpy()
    S0 = np.array([float(p.S0) for p in pr.problems])
    nrmse = np.sqrt(np.mean((sp - ep) ** 2, axis=1)) / S0
    cn = counts.cpu().numpy()
    return {"shots_per_instance": shots, "instances": batch,
            "shots_per_s": batch * shots / (sample_ms * 1e-3),
            "sample_ms": sample_ms, "shot_price_ms": shot_ms, "exact_observable_readout_ms": exact_ms,
            "sampler_roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_TFLOPS,
                                 "unit": "TFLOP/s (FP64 vector)", "frac": achieved / FP64_VECTOR_TFLOPS,
                                 "traffic": profiled_traffic("k_sample", SAMPLE_SOURCES),
                                 "traffic_per": PROFILED_TRAFFIC["k_sample"]["per"]},
            "shots_on_readout_strikes_frac": float(cn.sum() / (batch * shots)),
            "shot_vs_exact_observable_nrmse_mean": float(nrmse.mean()),
            "shot_vs_exact_observable_nrmse_max": float(nrmse.max()),
            "status_errors": {"sample": int((st.cpu().numpy() != 0).sum()),
                              "shot": int((st_shot.cpu().numpy() != 0).sum())}}


def _bs_call(S0, K, r, q, T, sigma):
    """Black–Scholes call (the reference the paper's NRMSE is measured against)."""
    from scipy import special
    sq = sigma * math.sqrt(T)
    d1 = (np.log(S0 / K) + (r - q + 0.5 * sigma * sigma) * T) / sq
    return S0 * math.exp(-q * T) * special.ndtr(d1) - K * math.exp(-r * T) * special.ndtr(d1 - sq)


def batched_sweep_point(cm, torch, n, batch, steps):
    """The headline workload's draws with n fixed: the SFFT chain (QTT build, zip-up,
    rounding, read-out of 4096 near-money strikes; operator cached) for the whole batch as
    one replayed HIP graph, and the dense complex64 FFT (all 2^n prices) on a subset of the
    same instances, both as grids/s; where the two cross is the batched crossover."""
    probs = W.heston_batch(batch, seed=20261203, n=n)
    nk = min(4096, 2 ** n)
    strikes = torch.from_numpy(np.stack([W.near_money(p, nk) for p in probs])).cuda()
    mpo = cm.MpoCache([n], 1e-9, 32, cm.CM_C64)
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32, mpo=mpo)
    pr.slots.update({"build": batch, "apply": min(batch, 1536), "round": batch})
    pr.capture(strikes)
    for _ in range(2):
        pr.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pr.replay()
    torch.cuda.synchronize()
    sfft_s = (time.perf_counter() - t0) / steps
    bad = int(sum((v != 0).sum() for v in pr.statuses().values()))
    # dense: as many instances as keep the price array near 4 GB, one launch each call
    nd = max(1, min(64, (1 << 30) // (2 ** n)))
    dprob = cm.pack_problems(probs[:nd], "cuda")
    dprices = torch.empty((nd, 2 ** n), dtype=torch.float32, device="cuda")
    dstat = torch.zeros(nd, dtype=torch.int32, device="cuda")
    dws = cm.Workspace("cuda")
    cm.cm_fft_price(dprob, nd, n, cm.CM_C64, None, 0, dprices, dstat, dws)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        cm.cm_fft_price(dprob, nd, n, cm.CM_C64, None, 0, dprices, dstat, dws)
    torch.cuda.synchronize()
    dense_s = (time.perf_counter() - t0) / (reps * nd)
    bad += int((dstat != 0).sum())
    del dprices, pr
    return {"n": n, "batch": batch, "sfft_grids_per_s": batch / sfft_s, "sfft_ms_per_step": sfft_s * 1e3,
            "dense_grids_per_s": 1.0 / dense_s, "dense_instances": nd,
            "sfft_over_dense": dense_s * batch / sfft_s, "status_errors": bad}


def paper_curves(cm, torch, ns, dense_max, tol=1e-10, mpo_tol=None, reps=3, shots=4096, build_tol=None):
    """Memory, maximal rank, run time and NRMSE against n on the paper's Black–Scholes grid
    (Section 4: S0 = 100, r = 0.05, sigma = 0.3, T = 0.5, alpha = 2.5, N = 2^(n-1),
    Delta_k = N^(-1/2)), FP64 throughout, one instance per run as in the paper:
      - sfft: operator construction (Q_n), QTT construction (x), and the Core (zip-up,
        rounding, read-out of the window strikes); memory = bytes of the final y train;
      - fft: the dense FFT with read-out of the same strikes (n <= dense_max); memory = the
        2^n complex array;
      - nrmse: over the grid strikes with 0.5 <= K/S0 <= 1.5 (at most 2^16 of them, evenly
        strided) against the Black–Scholes formula (Eq. error_measure);
      - qft: the observable arm (Section 2.2) from the same y train: the statevector NRMSE
        (exact probabilities, Eq. qft_observable_price with p_hat = p) and the NRMSE of the
        shot estimator with `shots` outcomes (seeded uniforms)."""
    rows = []
    mpo_tol = tol / 10 if mpo_tol is None else mpo_tol
    for n in ns:
        p = W.paper_bs_grid(n)
        M = 2 ** n
        lam = 2.0 * math.pi / (M * p.eta)
        u_lo = max(0, math.ceil((math.log(50.0) - p.k0) / lam))
        u_hi = min(M - 1, math.floor((math.log(150.0) - p.k0) / lam))
        u = np.arange(u_lo, u_hi + 1, dtype=np.int64)
        if len(u) > 65536:
            u = u[np.linspace(0, len(u) - 1, 65536).round().astype(np.int64)]
        # the exact grid strikes k0 + 2 pi u / (M eta), formed in extended precision: the
        # grid's k0 is ~2^(n/2) from the money, so rounding lambda first would move the strikes
        two_pi = np.longdouble(2) * np.arccos(np.longdouble(-1))
        K = np.exp((np.longdouble(p.k0) + two_pi / (np.longdouble(M) * np.longdouble(p.eta))
                    * u.astype(np.longdouble)).astype(np.float64))
        ref = _bs_call(100.0, K, 0.05, 0.0, 0.5, 0.3)
        sd = torch.from_numpy(u[None, :]).cuda()

        def timed(fn):
            best = float("inf")
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            return best

        box = {}
        t_op = timed(lambda: box.__setitem__("mpo", cm.MpoCache([n], mpo_tol, 64, cm.CM_C128)))
        pr = cm.SfftPricer([p], cm.CM_C128, tol=tol, cap=64, mpo=box["mpo"], build_tol=build_tol)
        prices = torch.empty((1, len(u)), dtype=torch.float64, device="cuda")
        t_x = timed(pr.build)
        t_core = timed(lambda: (pr.apply(), pr.round(), pr.read(sd, prices)))
        got = prices.cpu().numpy()[0]
        st = pr.statuses()
        yr = pr.y.ranks[0, : n + 1].cpu().numpy().astype(np.int64)
        row = {"n": n, "strikes": int(len(u)), "tol": tol, "mpo_tol": mpo_tol, "build_tol": pr.build_tol,
               "mpo_max_rank": int(box["mpo"].w.ranks[n, : n + 1].max().item()),
               "sfft": {"construct_operator_s": t_op, "construct_x_s": t_x, "core_s": t_core,
                        "total_s": t_op + t_x + t_core,
                        "memory_MB": float((yr[:-1] * 2 * yr[1:]).sum() * 16 / 1e6),
                        "max_rank": int(yr.max()), "x_max_rank": int(pr.x.ranks[0, : n + 1].max().item()),
                        "nrmse": float(np.sqrt(np.mean((got - ref) ** 2)) / 100.0),
                        "status": {k: int(v[0]) for k, v in st.items()}}}
        obs = torch.empty((1, len(u)), dtype=torch.float64, device="cuda")
        cm.cm_readout_observable(pr.y, pr.prob, sd, len(u), obs)
        g = torch.Generator(device="cuda")
        g.manual_seed(1000 + n)
        U = torch.rand((1, n, shots), dtype=torch.float64, device="cuda", generator=g)
        smp = torch.empty((1, shots), dtype=torch.int64, device="cuda")
        nrm = torch.empty(1, dtype=torch.float64, device="cuda")
        cnt = torch.empty((1, len(u)), dtype=torch.int32, device="cuda")
        spx = torch.empty((1, len(u)), dtype=torch.float64, device="cuda")
        qst = torch.zeros(1, dtype=torch.int32, device="cuda")
        cm.cm_sample_outcomes(pr.y, U, shots, smp, nrm, qst, cm.Workspace())
        cm.cm_shot_prices(pr.prob, 1, nrm, smp, shots, sd, len(u), cnt, spx, qst)
        row["qft"] = {"statevector_nrmse": float(np.sqrt(np.mean((obs.cpu().numpy()[0] - ref) ** 2)) / 100.0),
                      "shots": shots,
                      "shot_nrmse": float(np.sqrt(np.mean((spx.cpu().numpy()[0] - ref) ** 2)) / 100.0),
                      "status": int(qst.item())}
        if n <= dense_max:
            dbox = {}
            t_fft = timed(lambda: dbox.__setitem__("r", cm.dense_prices([p], cm.CM_C128, strikes=sd)))
            dgot = dbox["r"][0].cpu().numpy()[0]
            row["fft"] = {"total_s": t_fft, "memory_MB": M * 16 / 1e6,
                          "nrmse": float(np.sqrt(np.mean((dgot - ref) ** 2)) / 100.0)}
        print(json.dumps(row), flush=True)
        rows.append(row)
    return rows


BF16_DENSE_TFLOPS = 2500.0

# HBM bytes per dispatch from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs recorded in
# profiles/traffic_pmc_heston4096_n24.md (fetch scaled by 2.0 and write by 1.0, the factors a
# 1 GiB device copy gives). A figure is reported only while the kernel's sources hash to the
# value they had when the counters were taken.
ZIPUP_SOURCES = ["paper_2607_28435_amd/csrc/cm_zipup.hip", "paper_2607_28435_amd/csrc/cm_tt.h",
                 "paper_2607_28435_amd/csrc/cm_linalg.h", "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
FFT_SOURCES = ["paper_2607_28435_amd/csrc/cm_fft.hip", "paper_2607_28435_amd/csrc/cm_cf.h",
               "paper_2607_28435_amd/csrc/cm_tt.h", "paper_2607_28435_amd/csrc/cm_linalg.h",
               "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
SAMPLE_SOURCES = ["paper_2607_28435_amd/csrc/cm_sample.hip", "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
BUILD_SOURCES = ["paper_2607_28435_amd/csrc/cm_qtt.hip", "paper_2607_28435_amd/csrc/cm_cf.h",
                 "paper_2607_28435_amd/csrc/cm_tt.h", "paper_2607_28435_amd/csrc/cm_linalg.h",
                 "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
ROUND_SOURCES = ["paper_2607_28435_amd/csrc/cm_round.hip", "paper_2607_28435_amd/csrc/cm_tt.h",
                 "paper_2607_28435_amd/csrc/cm_linalg.h", "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
READ_SOURCES = ["paper_2607_28435_amd/csrc/cm_readout.hip", "paper_2607_28435_amd/csrc/cm_cf.h",
                "paper_2607_28435_amd/csrc/cm_tt.h", "paper_2607_28435_amd/csrc/cm_linalg.h",
                "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
MLP_SOURCES = ["paper_2607_28435_amd/csrc/cm_mlp.hip", "paper_2607_28435_amd/csrc/cm_internal.h", "include/cm.h"]
_F = 1.9999246625669753   # FETCH_SIZE scale of the 1 GiB copy (chain runs)
_FS = 1.999924424166386  # the same for the surrogate runs
PROFILED_TRAFFIC = {
    "k_zipup": {"sha": "e7e1d79ec8558963", "bytes": (199956.9 * _F + 849972.8) * 1024,
                "per": "launch (4096 instances, n=24, 1536 workgroups)"},
    "build": {"sha": "9ae1b95f36b0a318", "bytes": ((37192.0 + 401323.2) * _F + 229858.3 + 816959.3) * 1024,
              "per": "build (k_build_qtt + k_build_round, 4096 instances, n=24)"},
    "k_tt_round": {"sha": "b814f698d2149b43", "bytes": (241047.6 * _F + 417431.9) * 1024,
                   "per": "launch (4096 instances, n=24, 4096 workgroups)"},
    "k_readout": {"sha": "a8120f97e9153a98", "bytes": ((787.8 + 105182.8 + 788.6) * _F + 131072.0) * 1024,
                  "per": "read-out (k_readout<8> + <16> + <32>, 4096 instances x 4096 strikes)"},
    "dense": {"sha": "9662f05dd5eaea99", "bytes": ((157.5 + 65631.0) * _F + 131080.25 + 65536.0) * 1024,
              "per": "grid (k_fft_first + k_fft_next, n=24)"},
    "k_sample": {"sha": "b563430d544ae401", "bytes": (3780258.8 * _F + 131072.0) * 1024,
                 "per": "launch (4096 instances x 4096 shots, n=24)"},
    "surrogate": {"sha": "60db21156adabfa7", "bytes": ((16041.5 + 16407.0) * _FS + 4096.0 + 8192.0) * 1024,
                  "per": "pass over 2^20 queries (k_mlp_fused + k_gate)"},
}


def _sources_sha(files):
    import hashlib
    m = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def profiled_traffic(name, files):
    rec = PROFILED_TRAFFIC[name]
    return rec["bytes"] if _sources_sha(files) == rec["sha"] else None


def surrogate_run(cm, torch, steps):
    """Surrogate (config 5): train on 2^22 SFFT samples (2^16 parameter sets x 64 k, training
    box 20 % wider than the trusted box), then 2^20 held-out queries (90 % in the trusted
    box, 10 % from a box enlarged by 20 %): gated prices vs the SFFT reference, accept rate, and
    network+gate throughput against batched SFFT pricing of the same queries."""
    from paper_2607_28435_amd.surrogate import Surrogate
    lo, hi = W.surrogate_box()
    t0 = time.perf_counter()
    s = Surrogate(lo, hi, seed=0)
    X, Y = s.training_set(2 ** 16, 64, seed=1001)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    info = s.fit(X, Y, steps=steps, batch=8192, lr=2e-3, log_every=max(1, steps // 20))
    t0 = time.perf_counter()
    cal = s.calibrate(2 ** 15, seed=4001)
    cal["seconds"] = time.perf_counter() - t0
    nq = 2 ** 20
    q = np.concatenate([W.surrogate_queries(nq - nq // 10, 5001), W.surrogate_queries(nq // 10, 5002, enlarge=0.2)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref_prices, st = s.query_prices(q)
    torch.cuda.synchronize()
    sfft_s = time.perf_counter() - t0
    res = s.price(q)
    acc = res["accept"]
    ok = acc & (st == 0)
    err = np.abs(res["price"] - ref_prices)
    # network + gate throughput on all queries (device-resident inputs)
    # (50 untimed calls first: the clocks ramp up over the first tens of milliseconds of load;
    # then the median of five rounds of ten calls)
    qd = torch.from_numpy(q.astype(np.float32)).cuda()
    for _ in range(50):
        s.predict(qd)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps, rounds = 10, []
    for _ in range(5):
        e0.record(stream)
        for _ in range(reps):
            s.predict(qd)
        e1.record(stream)
        torch.cuda.synchronize()
        rounds.append(e0.elapsed_time(e1) * 1e-3 / reps)
    net_s = float(np.median(rounds))
    flops = 2.0 * 199681 * nq          # algorithmic (one multiply-add per weight per query)
    executed = flops + 2.0 * 3 * 65536 * nq   # the activation split runs the 256x256 layers twice
    ach = flops / net_s / 1e12
    # inputs (7 floats) read and network output written by the network; inputs and output
    # read, price and accept written by the gate
    algo_bytes = float(nq) * (4 * 8 + 4 * 10)
    tr = profiled_traffic("surrogate", MLP_SOURCES)
    return {"train_samples": int(len(Y)), "train_steps": info["steps"], "train_s": info["seconds"],
            "data_gen_s": gen_s, "final_train_loss": info["final_loss"], "gate_calibration": cal,
            "eval_queries": nq, "accept_rate": float(acc.mean()), "in_box_accept_rate": float(acc[:nq - nq // 10].mean()),
            "in_gate_max_abs_err_over_S0": float(err[ok].max()) if ok.any() else None,
            "in_gate_p999_abs_err_over_S0": float(np.quantile(err[ok], 0.999)) if ok.any() else None,
            "sfft_reference_failures": int((st != 0).sum()),
            "queries_per_s": nq / net_s, "sfft_queries_per_s": nq / sfft_s, "speedup_vs_sfft": sfft_s / net_s,
            "roofline": {"kernel": "k_mlp_fused + k_gate", "bound": "mfma",
                         "achieved": ach, "peak": BF16_DENSE_TFLOPS, "unit": "TFLOP/s",
                         "frac": ach / BF16_DENSE_TFLOPS, "executed_tflops": executed / net_s / 1e12,
                         "algorithmic_bytes": algo_bytes, "traffic": tr,
                         "traffic_per": PROFILED_TRAFFIC["surrogate"]["per"],
                         "traffic_over_algorithmic": (tr / algo_bytes) if tr else None}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2607_28435_amd as cm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.sweep:
        for n in args.sweep_list:
            print(json.dumps(batched_sweep_point(cm, torch, n, args.batch, args.steps)), flush=True)
        return
    if args.curves:
        ns = args.curves_list if args.curves_list else list(range(args.curves_n[0], args.curves_n[1] + 1))
        paper_curves(cm, torch, ns, args.curves_dense_max, tol=args.curves_tol, mpo_tol=args.curves_mpo_tol,
                     shots=args.curves_shots, build_tol=args.curves_build_tol)
        return
    dev = "cuda"
    if args.copy_calibration:
        a = torch.ones(2 ** 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    stream = torch.cuda.current_stream()
    probs = W.heston_batch(args.batch, seed=20261203, n=args.n)
    nk = 4096
    strikes = torch.from_numpy(np.stack([W.near_money(p, nk) for p in probs])).to(dev)
    prices = torch.empty((args.batch, nk), dtype=torch.float64, device=dev)

    t0 = time.perf_counter()
    mpo = cm.MpoCache([args.n], 1e-9, 32, cm.CM_C64)
    torch.cuda.synchronize()
    mpo_s = time.perf_counter() - t0
    pr = cm.SfftPricer(probs, cm.CM_C64, tol=1e-8, cap=32, mpo=mpo)
    # persistent-workgroup counts of the three sweep ops, timed on this batch (untimed)
    slots = {k: None for k in ("build", "apply", "round")}
    if args.autotune:
        slots = cm.autotune_slots(pr, strikes, candidates=SLOT_CANDIDATES, reps=2)
    elif not args.default_slots:
        slots = dict(zip(("build", "apply", "round"), args.slots))
        pr.slots.update(slots)

    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("build", "apply", "round", "read")}
    acc = {k: 0.0 for k in ev}

    def step(timed):
        if timed:
            ev["build"][0].record(stream)
        pr.build()
        if timed:
            ev["build"][1].record(stream)
            ev["apply"][0].record(stream)
        pr.apply()
        if timed:
            ev["apply"][1].record(stream)
            ev["round"][0].record(stream)
        pr.round()
        if timed:
            ev["round"][1].record(stream)
            ev["read"][0].record(stream)
        pr.read(strikes, prices)
        if timed:
            ev["read"][1].record(stream)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # per-stage times on eager steps
    for _ in range(args.steps):
        step(True)
        torch.cuda.synchronize()
        for k in ev:
            acc[k] += ev[k][0].elapsed_time(ev[k][1])
    # the timed region: the whole chain as one HIP graph, replayed
    if args.no_graph:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(False)
        torch.cuda.synchronize()
    else:
        pr.capture(strikes)
        for _ in range(max(1, args.warmup)):
            pr.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pr.replay()
        torch.cuda.synchronize()
        prices = pr.graph_prices
    sfft_s = (time.perf_counter() - t0) / args.steps
    sfft_gps = args.batch / sfft_s
    stat = pr.statuses()
    bad = {k: int((v != 0).sum()) for k, v in stat.items()}

    # dense baseline on a subset of the same problems (all 2^n prices per instance), timed right
    # after the SFFT chain so that both run under the same conditions
    nd = min(args.dense_instances, args.batch)
    dprob = cm.pack_problems(probs[:nd], dev)
    dprices = torch.empty((nd, 2 ** args.n), dtype=torch.float32, device=dev)
    dstat = torch.zeros(nd, dtype=torch.int32, device=dev)
    dws = cm.Workspace(dev)
    cm.cm_fft_price(dprob, nd, args.n, cm.CM_C64, None, 0, dprices, dstat, dws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 4
    e0.record(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        cm.cm_fft_price(dprob, nd, args.n, cm.CM_C64, None, 0, dprices, dstat, dws)
    e1.record(stream)
    torch.cuda.synchronize()
    dense_s = (time.perf_counter() - t0) / (reps * nd)
    dense_ms_ev = e0.elapsed_time(e1) / (reps * nd)
    M = 2 ** args.n
    dense_gps = 1.0 / dense_s
    dense_bytes = 8 * M + (8 * M + 4 * M) if args.n > 14 else 4 * M   # pass-1 write, pass-2 read + price write
    dense_gbs = dense_bytes / (dense_ms_ev * 1e-3) / 1e9
    # the same grids four instances per launch group (a workspace sized for it): the pass
    # buffers (4 x 134 MB at n = 24) exceed the 256 MB Infinity Cache, so the intermediate
    # makes a real DRAM round trip, unlike one instance per launch
    group = 4
    dws4 = cm.Workspace(dev)
    dws4.get(cm.cm_workspace_bytes(cm.CM_OP_FFT_PRICE, nd, args.n, 0, cm.CM_C64) + 8 * M * (group - 1))
    cm.cm_fft_price(dprob, nd, args.n, cm.CM_C64, None, 0, dprices, dstat, dws4)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        cm.cm_fft_price(dprob, nd, args.n, cm.CM_C64, None, 0, dprices, dstat, dws4)
    e1.record(stream)
    torch.cuda.synchronize()
    dense_dram_ms = e0.elapsed_time(e1) / (reps * nd)
    dense_dram_gbs = dense_bytes / (dense_dram_ms * 1e-3) / 1e9
    del dws4

    mpo_table = None
    if not args.no_mpo_table:
        mpo_table = mpo_table_run(cm, torch)
    qft = None
    if not args.no_qft:
        qft = qft_run(cm, torch, pr, strikes, args.shots, args.steps)

    # ranks for the flop models
    xr = pr.x.ranks.cpu().numpy()
    yr = pr.y.ranks.cpu().numpy()
    wr = mpo.w.ranks[args.n].cpu().numpy()
    # zip-up output ranks before rounding: rerun apply once (not timed) to read them
    pr.apply()
    torch.cuda.synchronize()
    yz = pr.y.ranks.cpu().numpy()
    pr.round()
    torch.cuda.synchronize()
    f32 = f64 = f_round = f_read = 0.0
    b_x = b_yz = b_y = 0
    s_host = strikes.cpu().numpy()
    read_cache = {}
    for b in range(args.batch):
        a32, a64 = zipup_flops(xr[b], wr, yz[b], args.n)
        f32 += a32
        f64 += a64
        f_round += round_flops(yz[b], yr[b], args.n)
        key = (tuple(yr[b, :args.n + 1]), s_host[b, 0])
        if key not in read_cache:
            read_cache[key] = readout_flops(yr[b], args.n, s_host[b])
        f_read += read_cache[key]
        b_x += core_elems(xr[b], args.n)
        b_yz += core_elems(yz[b], args.n)
        b_y += core_elems(yr[b], args.n)
    es = 8   # complex64 bytes
    ms = {k: acc[k] / args.steps for k in acc}
    B = args.batch
    stage_rooflines = {
        "build": alu_roofline("k_build_qtt + k_build_round (cm_build_qtt)", ms["build"], 0.0, SURVEY_BUILD_F64 * B,
                              es * b_x + 128 * B, "build", BUILD_SOURCES,
                              extra={"flops_model": "scope-table estimate, 3e6 FP64 per grid"}),
        "zipup": alu_roofline("k_zipup (cm_sfft_apply)", ms["apply"], f32, f64, es * (b_x + b_yz), "k_zipup",
                              ZIPUP_SOURCES, extra={
                                  "flops_model": "rank-exact (zipup_flops)",
                                  "frac_scope_formula": ((SURVEY_ZIPUP_F32 / (FP32_VECTOR_TFLOPS * 1e12) +
                                                          SURVEY_ZIPUP_F64 / (FP64_VECTOR_TFLOPS * 1e12)) * B /
                                                         (ms["apply"] * 1e-3))}),
        "round": alu_roofline("k_tt_round (cm_tt_round)", ms["round"], 0.0, f_round, es * (b_yz + b_y),
                              "k_tt_round", ROUND_SOURCES, extra={"flops_model": "rank-exact (round_flops)",
                                     "frac_scope_formula": SURVEY_ROUND_F64 * B / (FP64_VECTOR_TFLOPS * 1e12) /
                                     (ms["round"] * 1e-3)}),
        "readout": alu_roofline("k_readout (cm_readout_prices)", ms["read"], f_read, 0.0,
                                es * b_y + 16 * nk * B, "k_readout", READ_SOURCES, extra={"flops_model": "rank-exact, shared suffixes "
                                                                              "(readout_flops)"}),
    }
    frac = stage_rooflines["zipup"]["frac"]
    achieved_tf = stage_rooflines["zipup"]["achieved"]

    ragged = None
    if not args.no_ragged:
        ragged = ragged_run(cm, torch, args.batch, nk, args.steps, parity=not args.no_parity)
    vg = None
    if not args.no_vg:
        vg = vg_run(cm, torch, args.batch, nk, args.steps, args.n, parity=not args.no_parity)
    surrogate = None
    if not args.no_surrogate:
        surrogate = surrogate_run(cm, torch, args.surrogate_steps)

    # price errors are taken against the oracle prices of the cpu_baseline leg (below)
    max_err = None
    dense_err = None

    out = {
        "metric": "strike grids/sec, batched SFFT vs dense FFT at n=24, max abs price err/S0",
        "value": sfft_gps,
        "unit": "strike grids/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sfft_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 contraction / f64 factorisation",
        "data": "synthetic seeded Heston parameter draws",
        "config": {"workload": f"batched Heston SFFT, {args.batch} instances, n={args.n} "
                               f"(M=2^{args.n}), eta=40/2^{args.n // 2}, tol 1e-8, {nk} read-out strikes",
                   "batch": args.batch, "n": args.n, "parallelism": "none (1 GPU)",
                   "slots": {k: (int(v) if v is not None else "default") for k, v in slots.items()}},
        "dense_fft_grids_per_s": dense_gps,
        "sfft_over_dense": sfft_gps / dense_gps,
        "max_abs_err_over_S0": max_err,
        "dense_max_abs_err_over_S0": dense_err,
        "stage_ms": {k: acc[k] / args.steps for k in acc},
        "eager_ms_per_step": sum(acc.values()) / args.steps,
        "ragged": ragged,
        "variance_gamma": vg,
        "qft_observable": qft,
        "mpo_table": mpo_table,
        "surrogate": surrogate,
        "mpo_build_s": mpo_s,
        "status_errors": bad,
        "ranks": {"x_max": int(xr[:, :args.n + 1].max()), "y_max": int(yr[:, :args.n + 1].max()),
                  "w_max": int(wr[:args.n + 1].max())},
        "roofline": {"kernel": "k_zipup (cm_sfft_apply)", "bound": "alu", "achieved": achieved_tf,
                     "peak": FP64_VECTOR_TFLOPS, "unit": "TFLOP/s", "frac": frac,
                     "traffic": profiled_traffic("k_zipup", ZIPUP_SOURCES),
                     "traffic_per": PROFILED_TRAFFIC["k_zipup"]["per"],
                     "note": "achieved = FP64-equivalent rate: (FP32 flops/157.3T + FP64 flops/78.6T)/time x 78.6T; "
                             "frac counts rank-exact flops (the gate); frac_scope_formula uses the scope table's "
                             "per-grid estimate",
                     "frac_scope_formula": stage_rooflines["zipup"]["frac_scope_formula"],
                     "flops_fp32": f32, "flops_fp64": f64},
        "stage_rooflines": stage_rooflines,
        "dense_roofline": {"kernel": "k_fft_first + k_fft_next", "bound": "hbm", "achieved": dense_gbs,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dense_gbs / HBM_PEAK_GBS,
                           "algorithmic_bytes": dense_bytes, "traffic": profiled_traffic("dense", FFT_SOURCES),
                           "traffic_per": PROFILED_TRAFFIC["dense"]["per"],
                           "note": "one instance per launch: its 134 MB intermediate stays in the 256 MB Infinity "
                                   "Cache between the passes"},
        "dense_dram_roofline": {"kernel": "k_fft_first + k_fft_next, 4 instances per launch group", "bound": "hbm",
                                "achieved": dense_dram_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": dense_dram_gbs / HBM_PEAK_GBS, "algorithmic_bytes": dense_bytes,
                                "ms_per_grid": dense_dram_ms,
                                "note": "pass buffers of 4 instances (537 MB) exceed the Infinity Cache: DRAM-resident"},
    }
    if not args.no_cpu_baseline:
        rec, priced = cpu_baseline(probs)
        out["cpu_baseline"] = rec
        if not args.no_parity:
            got = prices.cpu().numpy()
            dgot = dprices.cpu().numpy()
            idx_host = strikes.cpu().numpy()
            errs, derrs = [], []
            for b, ref in priced:
                sel = idx_host[b]
                errs.append(np.abs(got[b] - ref[sel]).max() / probs[b].S0)
                if b < nd:
                    derrs.append(np.abs(dgot[b, sel] - ref[sel]).max() / probs[b].S0)
            out["max_abs_err_over_S0"] = float(max(errs))
            out["dense_max_abs_err_over_S0"] = float(max(derrs)) if derrs else None
            out["err_sample"] = f"{len(priced)} instance(s) x {nk} strikes against the oracle's dense prices"
            for leg in (ragged, vg):
                if leg and leg.get("_parity"):
                    leg["max_abs_err_over_S0"], _ = oracle_errors(leg["_parity"])
    for leg in (ragged, vg):
        if leg:
            leg.pop("_parity", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
