#!/usr/bin/env python
"""Throughput of SZx compression and decompression on one MI355X.

Workload: a 100x500x500 float32 field in the shape of the paper's Hurricane
fields (synthetic: k^-5/3 Gaussian random field with 20 % exact-zero regions),
value-range relative bounds 1e-2, 1e-3 and 1e-4, block size 128.

One step = for each of the three bounds, compress the field and decompress the
stream (every kernel of both directions, including the global range pass of
the relative bound). Inputs and outputs rotate over several copies so that the
256 MB last-level cache cannot serve a step from the previous step's data.
The steps are replayed from HIP graphs captured once per copy (the C ABI is
asynchronous and allocation-free, so a whole step captures); --eager launches
them directly instead.

Prints one JSON line. `value` is the round-trip throughput in GB/s of
uncompressed bytes: bytes compressed in the step divided by the time of the
step (compress + decompress). `detail.per_bound` holds, per bound, compress
and decompress GB/s, their fractions of the HBM peak by uncompressed and by
algorithmic bytes, the ratio, max error and PSNR (eq. (7)), block fractions,
K and code histograms and the error-control ladder's outcomes;
`detail.kernels` the per-kernel durations. The default run also measures the
2^28 float64 state vector the same way (`detail.state_2p28_float64`).
`roofline` is the dominant kernel's algorithmic bytes per launch over its
average launch duration (HIP events on its stream during a second,
instrumented timed region). `cpu_baseline` is the CPU oracle on the same
field and bounds: all cores of the affinity mask at once (one process per
core on disjoint block ranges), with the single-thread figure beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BLOCK = 128
# bench fields: the headline is turbulence; the others are for design measurements
FIELDS = {
    "turbulence": dict(shape=(100, 500, 500), bounds=(1e-2, 1e-3, 1e-4),
                 desc="100x500x500 float32 turbulence field with 20% zero regions"),
    "state": dict(shape=(1 << 28,), bounds=(1e-3, 1e-5),
                  desc="2^28 float64 state vector (exp-decaying complex amplitudes)"),
    "sphere": dict(shape=(1800, 3600), bounds=(1e-3, 1e-5), desc="1800x3600 float32 spherical-harmonic field"),
    "sines": dict(shape=(1 << 20,), bounds=(1e-3,), desc="2^20 float32 sum of sines"),
}
BOUNDS = FIELDS["turbulence"]["bounds"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--eager", action="store_true", help="launch directly instead of graph replay")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-state", action="store_true", help="skip the 2^28 float64 field of the default run")
    ap.add_argument("--profile", action="store_true",
                    help="short eager run for profilers: no CPU baseline, no instrumented pass, plus a plain 256 MiB copy whose HBM counters scale the others")
    ap.add_argument("--io-dir", type=str, default=None, help="io: directory for the stream files (default: a new temporary one)")
    ap.add_argument("--shards", type=str, default="2,4,8", help="shard: shard counts of the state vector")
    ap.add_argument("--field", type=str, default="turbulence", choices=sorted(FIELDS) + ["batch", "serve", "io", "shard"],
                    help="batch: the many-field batch (batched launches vs per-field calls); "
                         "serve: the serving loop (continuous batching vs serial FIFO)")
    ap.add_argument("--batch-fields", type=int, default=4096, help="batch: number of fields")
    ap.add_argument("--tune", action="store_true", help="batch: autotune the encode geometry first")
    ap.add_argument("--cpu-sample-fields", type=int, default=48, help="batch: fields the oracle runs on")
    ap.add_argument("--serve-requests", type=int, default=2000, help="serve: requests per load level")
    ap.add_argument("--serve-slots", type=int, default=4, help="serve: streams of the batching server")
    ap.add_argument("--serve-max-batch", type=int, default=64, help="serve: requests per launch group")
    ap.add_argument("--serve-budget-gib", type=int, default=64, help="serve: HBM budget of the server")
    return ap.parse_args()


def kernel_bytes(name, n, w, nblk, n_nc, mid_total, b=BLOCK):
    """Algorithmic HBM bytes of one launch of each kernel (reads + writes),
    from the sizes of the arrays each kernel must touch once."""
    codes = n_nc * (b // 4)
    tblk = 64 if w == 4 else 32  # blocks per encode tile at b = 128 (32 KiB of input)
    ntile = -(-nblk // tblk)
    ndtile = -(-nblk // (tblk // 2))  # decode tiles: 16 KiB of input
    if name == "k_stats":  # values in; per-block extrema out
        return n * w + nblk * 2 * w
    if name == "k_classify":  # extrema in; mu, state bits, plan bytes, tile ranks out
        return nblk * 2 * w + nblk * w + nblk / 8 + nblk + 8 * ntile
    if name == "k_encode":  # mu, plan bytes, tile ranks, non-constant values in; K, codes, mid out
        return nblk * w + nblk + 8 * ntile + n_nc * b * w + n_nc + codes + mid_total
    if name == "k_dindex":  # state bits, K, codes in; tile index out
        return nblk / 8 + n_nc + codes + 16 * ndtile
    if name == "k_decode":  # index, state, mu, K, codes, mid in; values out
        return 16 * ndtile + nblk / 8 + nblk * w + n_nc + codes + mid_total + n * w
    return 0


def source_hash():
    """sha256 over the HIP sources, as recorded beside the counter summaries."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2201_13020_amd", "csrc", "*"))):
        h.update(os.path.basename(p).encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()


def recorded_traffic(kernel, tag="turbulence"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs, scaled by a plain copy), or None
    when the summary is missing or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "source_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if fields.get("source_sha256") != source_hash():
        return None
    table = json.loads(fields.get("traffic_bytes_per_launch", "{}"))
    for k, v in table.items():
        if k.split("<")[0] == kernel:
            return int(v)
    return None


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo ("unknown" if absent)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores():
    """CPUs this process may run on (its affinity mask), at most 16: the
    share of the host that one GPU's job may use."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_worker(task):
    """One CPU worker of the all-cores leg: compress + decompress its slice of
    the field at every bound with the oracle until `seconds` have passed.
    Returns (bytes processed, compress s, decompress s)."""
    x, bounds, block, seconds, cpu = task
    if cpu is not None:
        try:
            os.sched_setaffinity(0, {cpu})
        except (AttributeError, OSError):
            pass
    sys.path.insert(0, ROOT)
    from oracle import szref
    tc = td = 0.0
    done = 0
    while done == 0 or tc + td < seconds:
        for eb in bounds:
            t0 = time.perf_counter()
            ref = szref.compress(x, eb, "rel", block)
            t1 = time.perf_counter()
            szref.decompress(ref)
            t2 = time.perf_counter()
            tc += t1 - t0
            td += t2 - t1
            done += x.nbytes
    return done, tc, td


def cpu_all_cores(x_np, bounds, seconds=8.0):
    """The oracle on P disjoint block-range slices of the field at once, one
    process per core of the affinity mask (a timing context: each slice takes
    its own relative bound and the streams are not joined)."""
    import multiprocessing as mp
    P = host_cores()
    flat = x_np.reshape(-1)
    nblk = -(-flat.size // BLOCK)
    cuts = [(nblk * i // P) * BLOCK for i in range(P + 1)]
    cuts[-1] = flat.size
    try:
        cpus = sorted(os.sched_getaffinity(0))[:P]
    except AttributeError:
        cpus = [None] * P
    tasks = [(flat[cuts[i]:cuts[i + 1]].copy(), bounds, BLOCK, seconds, cpus[i]) for i in range(P)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(P) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, tasks)
        wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    return {"value": round(done / wall / 1e9, 4), "cores": P, "seconds": round(wall, 3),
            "sample": f"{P} processes, one per core, each on a contiguous 1/{P} block range of the field, "
                      f"compress + decompress at every bound repeated for about {seconds:.0f} s"}


def to_keys(s, W):
    """Signed integers whose order is IEEE totalOrder, from the bit patterns s
    (int32/int64 tensor) of W-bit floats; the map is its own inverse."""
    return s ^ ((s >> (W - 1)) & ((1 << (W - 1)) - 1))


def stream_stats(x, out, size):
    """Block outcomes of one compressed stream (device tensors: the field x,
    the stream buffer out, its size): fractions of constant, coded and raw
    blocks, histograms of the kept bits K and of the 2-bit codes, and the
    escalations of the error-control ladder, counted against eq. (4)'s first
    rung K0 computed here from each block's extrema (a measurement only: the
    stream is what the kernels wrote)."""
    import struct
    import torch
    hdr = out[:96].cpu().numpy().tobytes()
    dt_code, b = hdr[5], struct.unpack_from("<I", hdr, 8)[0]
    e_bits, nblk, n_nc, mid_total = struct.unpack_from("<4Q", hdr, 64)
    w = 4 if dt_code == 0 else 8
    W, E, BIAS = (32, 8, 127) if w == 4 else (64, 11, 1023)
    MANT = W - 1 - E
    idt = torch.int32 if w == 4 else torch.int64

    def a16(v):
        return (v + 15) & ~15
    st_off = 96
    mu_off = a16(st_off + (nblk + 7) // 8)
    k_off = a16(mu_off + nblk * w)
    c_off = a16(k_off + n_nc)
    state = out[st_off:st_off + (nblk + 7) // 8]
    bits = ((state.to(torch.int32).unsqueeze(1) >> torch.arange(8, device=out.device)) & 1).reshape(-1)[:nblk]
    K = out[k_off:k_off + n_nc].to(torch.int64)
    raw = K == 0xFF
    n_raw = int(raw.sum())
    n = x.numel()
    # codes of coded blocks over their valid values
    codes = out[c_off:c_off + n_nc * (b // 4)].reshape(n_nc, b // 4).to(torch.int32)
    shifts = torch.tensor([6, 4, 2, 0], device=out.device, dtype=torch.int32)
    cv = ((codes.unsqueeze(2) >> shifts) & 3).reshape(n_nc, b)
    nc_idx = torch.nonzero(bits).reshape(-1)
    valid = torch.ones_like(cv, dtype=torch.bool)
    if n % b and n_nc and int(nc_idx[-1]) == nblk - 1:
        valid[-1, n % b:] = False
    valid &= ~raw.unsqueeze(1)
    code_hist = torch.bincount(cv[valid].reshape(-1).to(torch.int64), minlength=4).tolist()
    K_hist = {int(k): int(c) for k, c in enumerate(torch.bincount(K, minlength=256).tolist()) if c}
    # first rung of every non-constant block from its extrema
    s = x.reshape(-1).view(idt)
    pad = nblk * b - n
    if pad:
        s = torch.cat([s, s[-1:].expand(pad)])
    key = to_keys(s.reshape(nblk, b), W)
    kn = key.min(1).values[nc_idx]
    kx = key.max(1).values[nc_idx]
    mn = to_keys(kn, W).view(x.dtype)
    mx = to_keys(kx, W).view(x.dtype)
    fin = torch.isfinite(mn) & torch.isfinite(mx)
    mu = 0.5 * mn + 0.5 * mx
    r = torch.maximum((mx - mu).abs(), (mn - mu).abs())

    def p_of(v_bits):
        f = (v_bits >> MANT) & ((1 << E) - 1)
        return torch.clamp(f, min=1) - BIAS
    e = torch.tensor([e_bits], dtype=idt, device=out.device)  # e >= 0: the sign bit is clear
    m0 = torch.clamp(p_of(r.view(idt)) - p_of(e), min=0)
    K0 = torch.clamp(1 + E + m0, max=W).to(torch.int64)
    coded = ~raw
    up1 = int((coded & fin & (K == K0 + 1) & (K0 < W)).sum())
    at0 = int((coded & fin & (K == K0)).sum())
    raw_fail = int((raw & fin).sum())
    return {
        "blocks": int(nblk),
        "constant_frac": round(1 - n_nc / max(nblk, 1), 6),
        "coded_frac": round((n_nc - n_raw) / max(nblk, 1), 6),
        "raw_frac": round(n_raw / max(nblk, 1), 6),
        "K_hist": K_hist,
        "code_hist": code_hist,
        "ladder": {"first_rung": at0, "second_rung_K0_plus_1": up1, "raw_by_failure": raw_fail,
                   "raw_non_finite": n_raw - raw_fail},
        "mid_bytes": int(mid_total),
    }


def quality(x, y, e_bits, w):
    """Max |x - x'| (and over e) and PSNR of eq. (7) over the finite values."""
    import math
    import struct
    import torch
    xd = x.reshape(-1).double()
    yd = y.reshape(-1).double()
    fin = torch.isfinite(xd)
    d = (yd - xd)[fin]
    mx = float(d.abs().max()) if d.numel() else 0.0
    mse = float((d * d).mean()) if d.numel() else 0.0
    rng = float(xd[fin].max() - xd[fin].min()) if d.numel() else 0.0
    e = struct.unpack("<f" if w == 4 else "<d", struct.pack("<Q", e_bits)[:w])[0]
    psnr = 20 * math.log10(rng / math.sqrt(mse)) if mse > 0 and rng > 0 else float("inf")
    return {"max_abs_err": mx, "max_err_over_e": (mx / e) if e > 0 else (0.0 if mx == 0 else float("inf")),
            "psnr_db": round(psnr, 3), "e": e}


def measure_field(name, args, dev, cpu_leg):
    """Compress + decompress one workload field at each of its bounds on the
    GPU: graph-replayed steps (the round-trip value), per-direction timings,
    per-kernel durations, whole-call algorithmic fractions, stream and
    quality statistics; with cpu_leg, the oracle's check and timing."""
    import struct
    import numpy as np
    import torch
    from paper_2201_13020_amd import synth, szx

    field = FIELDS[name]
    bounds = field["bounds"]
    shape = field["shape"]
    t0 = time.perf_counter()
    x_np = synth.make(name)
    _log(f"{name}: generated {x_np.nbytes / 1e6:.0f} MB in {time.perf_counter() - t0:.1f} s")
    n = x_np.size
    w = x_np.itemsize
    nbytes = n * w
    tdt = torch.float32 if w == 4 else torch.float64
    # copies so that the inputs exceed the 256 MB last-level cache
    C = max(1, args.copies if nbytes < (1 << 30) else 2)
    xs = [torch.from_numpy(x_np).to(dev) for _ in range(C)]
    cap = szx.compress_bound(tdt, shape, 1e-3, "rel", BLOCK)
    wsz = szx.workspace_size(tdt, shape, 1e-3, "rel", BLOCK)
    outs = {eb: [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in range(C)] for eb in bounds}
    sizes = {eb: [torch.zeros(1, dtype=torch.uint64, device=dev) for _ in range(C)] for eb in bounds}
    ys = [torch.empty(n, dtype=tdt, device=dev) for _ in range(C)]
    stat = torch.zeros(1, dtype=torch.uint32, device=dev)
    ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    expected = dict(dtype=tdt, dims=shape, block=BLOCK)

    def step(c, timed_ops=None):
        for eb in bounds:
            if timed_ops is not None:
                timed_ops[eb][0].record()
            szx.compress(xs[c], eb, "rel", BLOCK, out=outs[eb][c], out_size=sizes[eb][c], ws=ws)
            if timed_ops is not None:
                timed_ops[eb][1].record()
            szx.decompress(outs[eb][c], cap, expected, out=ys[c], status=stat, ws=ws)
            if timed_ops is not None:
                timed_ops[eb][2].record()

    # stream statistics and reconstruction quality, one bound at a time
    stream_len, ratios, per_bound = {}, {}, {}
    for eb in bounds:
        szx.compress(xs[0], eb, "rel", BLOCK, out=outs[eb][0], out_size=sizes[eb][0], ws=ws)
        szx.decompress(outs[eb][0], cap, expected, out=ys[0], status=stat, ws=ws)
        torch.cuda.synchronize()
        assert int(stat.cpu().view(torch.int32).item()) == 0, f"{name} eb={eb}: decoder status"
        stream_len[eb] = int(sizes[eb][0].cpu().view(torch.int64).item())
        ratios[eb] = nbytes / stream_len[eb]
        e_bits = struct.unpack_from("<Q", outs[eb][0][:96].cpu().numpy().tobytes(), 64)[0]
        q = quality(xs[0], ys[0], e_bits, w)
        assert q["max_err_over_e"] <= 1.0, f"{name} eb={eb}: error above the bound"
        per_bound[eb] = {"quality": q, "blocks": stream_stats(xs[0], outs[eb][0], sizes[eb][0])}
    _log(f"{name}: ratios {', '.join(f'{r:.3f}' for r in ratios.values())}")

    # correctness against the CPU oracle (also the single-thread CPU timing)
    cpu = None
    if cpu_leg:
        from oracle import szref
        step(0)
        torch.cuda.synchronize()
        try:
            aff = os.sched_getaffinity(0)
            os.sched_setaffinity(0, {min(aff)})
        except (AttributeError, OSError):
            aff = None
        # the whole workload, repeated until about 10 s of CPU time (the
        # first pass also checks the GPU results against the oracle)
        t_c = t_d = 0.0
        passes = 0
        try:
            while passes == 0 or (t_c + t_d < 10.0 and passes < 64):
                for eb in bounds:
                    t0 = time.perf_counter()
                    ref = szref.compress(x_np, eb, "rel", BLOCK)
                    t1 = time.perf_counter()
                    yref = szref.decompress(ref)
                    t2 = time.perf_counter()
                    t_c += t1 - t0
                    t_d += t2 - t1
                    if passes == 0:
                        gpu_stream = outs[eb][0][: stream_len[eb]].cpu().numpy()
                        assert gpu_stream.size == ref.size and np.array_equal(gpu_stream, ref), \
                            f"GPU stream differs from the oracle at eb={eb}"
                if passes == 0:
                    y_last = ys[0].cpu().numpy()
                    udt = np.uint32 if w == 4 else np.uint64
                    assert np.array_equal(y_last.view(udt), yref.ravel().view(udt)), \
                        "GPU decode differs from the oracle"
                passes += 1
        finally:
            if aff is not None:
                os.sched_setaffinity(0, aff)
        done = passes * len(bounds) * nbytes
        cpu = {"single_thread": {
            "value": round(done / (t_c + t_d) / 1e9, 4),
            "compress_MBps": round(done / t_c / 1e6, 1), "decompress_MBps": round(done / t_d / 1e6, 1),
            "passes": passes, "seconds": round(t_c + t_d, 3)}}
        _log(f"{name}: oracle single thread matched; {cpu['single_thread']}")
        cpu["all_cores"] = cpu_all_cores(x_np, bounds)
        _log(f"{name}: oracle all cores {cpu['all_cores']}")

    # graphs, one per copy
    graphs = None
    if not args.eager and not args.profile:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for c in range(C):
                step(c)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graphs = []
        for c in range(C):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                step(c)
            graphs.append(g)
        torch.cuda.synchronize()

    def run(c):
        if graphs is not None:
            graphs[c].replay()
        else:
            step(c)

    for i in range(args.warmup):
        run(i % C)
    torch.cuda.synchronize()
    # timed region
    t0 = time.perf_counter()
    for i in range(args.steps):
        run(i % C)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert int(stat.cpu().view(torch.int32).item()) == 0
    res = {"name": name, "desc": field["desc"], "bounds": bounds, "n": n, "w": w, "nbytes": nbytes, "copies": C,
           "launch": "eager" if graphs is None else "hip graph replay",
           "ms_per_step": elapsed * 1e3 / args.steps,
           "value": len(bounds) * nbytes / (elapsed / args.steps) / 1e9, "cpu": cpu}
    if args.profile:
        return res

    facts = {}
    for eb in bounds:
        facts[eb] = struct.unpack_from("<3Q", outs[eb][0][:96].cpu().numpy().tobytes(), 72)
    # per-direction timings: events between the calls on the same stream
    ev = {eb: [torch.cuda.Event(enable_timing=True) for _ in range(3)] for eb in bounds}
    tc = {eb: 0.0 for eb in bounds}
    td = {eb: 0.0 for eb in bounds}
    for i in range(args.steps):
        step(i % C, ev)
        torch.cuda.synchronize()
        for eb in bounds:
            tc[eb] += ev[eb][0].elapsed_time(ev[eb][1])
            td[eb] += ev[eb][1].elapsed_time(ev[eb][2])
    detail = {}
    for eb in bounds:
        c_ms = tc[eb] / args.steps
        d_ms = td[eb] / args.steps
        nblk, n_nc, mid_total = facts[eb]
        C_bytes = stream_len[eb]
        f_nc = n_nc / max(nblk, 1)
        alg_c = nbytes * (1 + f_nc) + C_bytes  # REL: the range pass reads all, the encoder re-reads non-constant blocks
        alg_d = C_bytes + nbytes
        detail[str(eb)] = {
            "ratio": round(ratios[eb], 4),
            "compress_GBps": round(nbytes / c_ms / 1e6, 1),
            "decompress_GBps": round(nbytes / d_ms / 1e6, 1),
            "compress_ms": round(c_ms, 4),
            "decompress_ms": round(d_ms, 4),
            "compress_hbm_frac_uncompressed": round(nbytes / c_ms / 1e6 / HBM_PEAK_GBPS, 4),
            "decompress_hbm_frac_uncompressed": round(nbytes / d_ms / 1e6 / HBM_PEAK_GBPS, 4),
            "compress_alg_bytes": int(alg_c),
            "decompress_alg_bytes": int(alg_d),
            "compress_hbm_frac_alg": round(alg_c / c_ms / 1e6 / HBM_PEAK_GBPS, 4),
            "decompress_hbm_frac_alg": round(alg_d / d_ms / 1e6 / HBM_PEAK_GBPS, 4),
            **per_bound[eb],
        }
    res["per_bound"] = detail

    # per-kernel durations with HIP events around each launch (same stream)
    szx.timing_enable(True)
    szx.timing_read()
    for i in range(args.steps):
        step(i % C)
    torch.cuda.synchronize()
    kt = szx.timing_read()
    szx.timing_enable(False)
    kernels = {}
    for kname, (cnt, ms) in kt.items():
        # each kernel runs once per bound per step: average algorithmic bytes over the bounds
        alg = sum(kernel_bytes(kname, n, w, *facts[eb]) for eb in bounds) / len(bounds)
        avg_ms = ms / cnt
        kernels[kname] = {"launches": cnt, "avg_us": round(avg_ms * 1e3, 2), "alg_bytes_per_launch": int(alg),
                          "achieved_GBps": round(alg / avg_ms / 1e6, 1) if alg else None}
    res["kernels"] = kernels
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (sharding over several GPUs is a design, not built)"}))
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.field == "batch":
        return bench_batch(args)
    if args.field == "serve":
        return bench_serve(args)
    if args.field == "io":
        return bench_io(args)
    if args.field == "shard":
        return bench_shard(args)
    dev = torch.device("cuda:0")
    cpu_leg = not args.no_cpu_baseline and not args.profile
    head = measure_field(args.field, args, dev, cpu_leg)
    bounds = head["bounds"]
    result = {
        "metric": "compress & decompress GB/s (uncompressed) and % of HBM peak; ratio",
        "value": round(head["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head["w"] == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{head['desc']}, REL {', '.join(map(str, bounds))}, block {BLOCK}; "
                               "one step = compress + decompress at each bound",
                   "global_batch": len(bounds), "elements": head["n"], "block": BLOCK,
                   "parallelism": "single GPU", "launch": head["launch"], "input_copies": head["copies"]},
    }
    if not args.profile:
        kernels = head["kernels"]
        result["detail"] = {"per_bound": head["per_bound"], "kernels": kernels}
        dom = max((k for k in kernels if kernels[k]["alg_bytes_per_launch"]),
                  key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
        kd = kernels[dom]
        result["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": kd["achieved_GBps"],
                              "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                              "frac": round(kd["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                              "traffic": recorded_traffic(dom, args.field),
                              "alg_bytes_per_launch": kd["alg_bytes_per_launch"], "avg_launch_us": kd["avg_us"]}
        if args.field == "turbulence" and not args.no_state:
            # the 2 GiB float64 field, timed in the same run (graph replay)
            st = measure_field("state", args, dev, False)
            sk = st["kernels"]
            sdom = max((k for k in sk if sk[k]["alg_bytes_per_launch"]),
                       key=lambda k: sk[k]["avg_us"] * sk[k]["launches"])
            result["detail"]["state_2p28_float64"] = {
                "workload": f"{st['desc']}, REL {', '.join(map(str, st['bounds']))}, block {BLOCK}",
                "round_trip_GBps": round(st["value"], 2), "ms_per_step": round(st["ms_per_step"], 4),
                "launch": st["launch"], "input_copies": st["copies"],
                "per_bound": st["per_bound"], "kernels": sk,
                "roofline": {"bound": "hbm", "kernel": sdom, "achieved": sk[sdom]["achieved_GBps"],
                             "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                             "frac": round(sk[sdom]["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                             "traffic": recorded_traffic(sdom, "state"),
                             "alg_bytes_per_launch": sk[sdom]["alg_bytes_per_launch"],
                             "avg_launch_us": sk[sdom]["avg_us"]}}
    cpu = head["cpu"]
    if cpu is not None:
        single, allc = cpu["single_thread"], cpu["all_cores"]
        result["cpu_baseline"] = {
            "value": allc["value"], "unit": "GB/s", "cores": allc["cores"], "kind": "oracle",
            "sample": f"{head['desc']}, REL {', '.join(map(str, bounds))}: {allc['sample']}; "
                      f"bytes compressed per second of compress + decompress, as for the GPU value",
            "cpu_model": cpu_model(),
            "single_thread": {"value": single["value"], "unit": "GB/s", "cores": 1,
                              "compress_MBps": single["compress_MBps"],
                              "decompress_MBps": single["decompress_MBps"],
                              "sample": f"whole workload {single['passes']} times on one pinned core, "
                                        f"{single['seconds']} s; the first pass matched the GPU byte for byte"},
            "seconds": allc["seconds"]}

    if args.profile:
        # a plain device copy of known size, to scale the HBM byte counters
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_batch(args):
    """Many fields of uneven sizes and both element types: one graph-replayed
    batch launch per direction against per-field calls (eager, and captured
    into one graph), every field's stream checked equal between the two and a
    sample against the oracle."""
    import ctypes
    import struct

    import numpy as np
    import torch
    from paper_2201_13020_amd import synth, szx, tune

    dev = torch.device("cuda:0")
    specs = synth.batch_specs(args.batch_fields)
    t0 = time.perf_counter()
    xs = [synth.batch_field(sp, dev) for sp in specs]
    torch.cuda.synchronize()
    _log(f"generated {len(xs)} fields in {time.perf_counter() - t0:.1f} s")
    nbytes = [x.numel() * x.element_size() for x in xs]
    total = sum(nbytes)
    by_dtype = {"float32": 0, "float64": 0}
    for sp, nb in zip(specs, nbytes):
        by_dtype[sp["dtype"]] += nb
    ebs = [sp["eb"] for sp in specs]
    dims = [sp["dims"] for sp in specs]
    tuned_from_cache = tune.apply_cache(block=BLOCK)

    cb = szx.compress_batch(xs, ebs, "rel", BLOCK, dims=dims)
    tuning = None
    if args.tune:
        res = tune.tune_batch(cb, by_dtype, BLOCK)
        tuning = {dt: {"encode_wgs": r[0], "ms": round(r[1], 4),
                       "candidates_ms": {str(k): round(v, 4) for k, v in r[2].items()}} for dt, r in res.items()}
        _log(f"tuned {tuning}")
    cb.run()
    torch.cuda.synchronize()
    lens = torch.stack(cb.sizes).cpu().view(torch.int64).reshape(-1).tolist()
    assert all(l > 0 for l in lens), "a batch field failed to compress"
    comp_total = sum(lens)
    heads = torch.stack([o[:96] for o in cb.outs]).cpu().numpy()
    exps = [szx.inspect(h.tobytes()) for h in heads]
    db = szx.decompress_batch(cb.outs, lens, exps)
    db.run()
    torch.cuda.synchronize()
    assert all(int(v) == 0 for v in torch.stack(db.statuses).cpu().view(torch.int32).reshape(-1)), "decode status"

    # per-field calls into their own buffers, parameter structs built before timing
    ws = torch.empty(max(szx.workspace_size(x.dtype, d, 1e-3, "rel", BLOCK) for x, d in zip(xs, dims)),
                     dtype=torch.uint8, device=dev)
    pf_out = [torch.empty_like(o) for o in cb.outs]
    pf_size = [torch.zeros(1, dtype=torch.uint64, device=dev) for _ in xs]
    pf_y = [torch.empty_like(y) for y in db.outs]
    pf_st = torch.zeros(1, dtype=torch.uint32, device=dev)
    cparams = [szx.make_params(x.dtype, d, eb, "rel", BLOCK) for x, d, eb in zip(xs, dims, ebs)]
    L = szx.lib()

    def per_field_compress():
        sh = szx._stream_handle(None)
        for i, x in enumerate(xs):
            rc = L.sz_compress(ctypes.byref(cparams[i]), x.data_ptr(), pf_out[i].data_ptr(), pf_out[i].numel(),
                               pf_size[i].data_ptr(), ws.data_ptr(), ws.numel(), sh)
            assert rc == 0, L.sz_last_error()

    def per_field_decompress():
        sh = szx._stream_handle(None)
        for i in range(len(xs)):
            rc = L.sz_decompress(cb.outs[i].data_ptr(), lens[i], ctypes.byref(cparams[i]), pf_y[i].data_ptr(),
                                 pf_y[i].numel() * pf_y[i].element_size(), pf_st.data_ptr(), ws.data_ptr(),
                                 ws.numel(), sh)
            assert rc == 0, L.sz_last_error()

    per_field_compress()
    per_field_decompress()
    torch.cuda.synchronize()
    same = all(torch.equal(cb.outs[i][:lens[i]], pf_out[i][:lens[i]]) for i in range(len(xs)))
    same = same and torch.stack(pf_size).cpu().view(torch.int64).reshape(-1).tolist() == lens
    same_y = all(torch.equal(db.outs[i].view(torch.uint8), pf_y[i].view(torch.uint8)) for i in range(len(xs)))
    assert same and same_y, "batch and per-field outputs differ"
    _log("batch output == per-field output for every field")

    def capture(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        torch.cuda.synchronize()
        return g

    g_c = capture(cb.run)
    g_d = capture(db.run)
    t0 = time.perf_counter()
    g_pfc = capture(per_field_compress)
    g_pfd = capture(per_field_decompress)
    _log(f"captured per-field graphs in {time.perf_counter() - t0:.1f} s")

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / steps

    steps, warm = args.steps, args.warmup
    for _ in range(warm):
        g_c.replay()
        g_d.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g_c.replay()
        g_d.replay()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    _log(f"timed {steps} batched steps: {ms_step:.3f} ms each")
    ms = {
        "batch_compress": timed(g_c.replay, steps, 2),
        "batch_decompress": timed(g_d.replay, steps, 2),
        "per_field_graph_compress": timed(g_pfc.replay, max(3, steps // 4), 1),
        "per_field_graph_decompress": timed(g_pfd.replay, max(3, steps // 4), 1),
        "per_field_eager_compress": timed(per_field_compress, 3, 1),
        "per_field_eager_decompress": timed(per_field_decompress, 3, 1),
    }
    gbps = {k: round(total / v / 1e6, 1) for k, v in ms.items()}
    _log(f"GB/s {gbps}")

    # kernel durations of the batched launches (HIP events around each launch)
    szx.timing_enable(True)
    szx.timing_read()
    for _ in range(steps):
        cb.run()
        db.run()
    torch.cuda.synchronize()
    kt = szx.timing_read()
    szx.timing_enable(False)
    alg = {}
    for i, x in enumerate(xs):
        nblk, n_nc, mid_total = struct.unpack_from("<3Q", heads[i].tobytes(), 72)
        for k in ("k_stats", "k_classify", "k_encode", "k_dindex", "k_decode"):
            alg[k] = alg.get(k, 0) + kernel_bytes(k, x.numel(), x.element_size(), nblk, n_nc, mid_total)
    kernels = {}
    for name, (cnt, kms) in kt.items():
        per_run_ms = kms / steps
        a = alg.get(name, 0)
        kernels[name] = {"launches_per_run": cnt // steps, "us_per_run": round(per_run_ms * 1e3, 1),
                         "alg_bytes_per_run": int(a), "achieved_GBps": round(a / per_run_ms / 1e6, 1) if a else None}
    dom = max((k for k in kernels if kernels[k]["alg_bytes_per_run"]), key=lambda k: kernels[k]["us_per_run"])
    kd = kernels[dom]

    cpu = None
    if not args.no_cpu_baseline and args.cpu_sample_fields > 0:
        from oracle import szref
        r = np.random.default_rng(5)
        pick = sorted(r.choice(len(xs), size=min(args.cpu_sample_fields, len(xs)), replace=False).tolist())
        hosts = [xs[i].cpu().numpy() for i in pick]
        # the sample, repeated until about 10 s of CPU time (the first pass
        # also checks the batch output against the oracle)
        tc = td = 0.0
        sb = 0
        passes = 0
        while passes == 0 or (tc + td < 10.0 and passes < 256):
            for i, xh in zip(pick, hosts):
                t1 = time.perf_counter()
                ref = szref.compress(xh, ebs[i], "rel", BLOCK)
                t2 = time.perf_counter()
                yref = szref.decompress(ref)
                t3 = time.perf_counter()
                tc += t2 - t1
                td += t3 - t2
                sb += xh.nbytes
                if passes == 0:
                    assert np.array_equal(cb.outs[i][:lens[i]].cpu().numpy(), ref), f"field {i} differs from the oracle"
                    udt = np.uint32 if xh.itemsize == 4 else np.uint64
                    yb = db.outs[i].cpu().numpy()
                    assert np.array_equal(yb.view(udt), yref.ravel().view(udt)), \
                        f"field {i} decode differs from the oracle"
            passes += 1
        cpu = {"value": round(sb / (tc + td) / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(pick)} fields of the batch drawn at random ({sb / passes / 2**20:.0f} MiB), "
                         f"compress + decompress each, {passes} times, single thread; matched the batch output "
                         f"byte for byte",
               "seconds": round(tc + td, 3)}
        _log(f"oracle sample of {len(pick)} fields matched")

    result = {
        "metric": "compress & decompress GB/s (uncompressed) and % of HBM peak; ratio",
        "value": round(total / ms_step / 1e6, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{len(xs)} fields, sizes lognormal 4 KiB-64 MiB (median 1 MiB), "
                               f"{100 * by_dtype['float64'] / total:.0f}% of bytes float64, 1-3 dims, REL "
                               "1e-2/1e-3/1e-4 per field, block 128; one step = batched compress + batched decompress",
                   "fields": len(xs), "bytes": total, "block": BLOCK, "parallelism": "single GPU",
                   "launch": "hip graph replay, one launch per pass and element type"},
        "detail": {
            "ratio": round(total / comp_total, 4),
            "ms": {k: round(v, 4) for k, v in ms.items()},
            "GBps_uncompressed": gbps,
            "hbm_frac_uncompressed": {k: round(v / HBM_PEAK_GBPS, 4) for k, v in gbps.items()},
            "batch_speedup_vs_per_field_graph": {
                "compress": round(ms["per_field_graph_compress"] / ms["batch_compress"], 2),
                "decompress": round(ms["per_field_graph_decompress"] / ms["batch_decompress"], 2)},
            "batch_speedup_vs_per_field_eager": {
                "compress": round(ms["per_field_eager_compress"] / ms["batch_compress"], 2),
                "decompress": round(ms["per_field_eager_decompress"] / ms["batch_decompress"], 2)},
            "kernels": kernels,
            "tuning": tuning,
            "tuned_entries_from_cache": tuned_from_cache,
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kd["achieved_GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(kd["achieved_GBps"] / HBM_PEAK_GBPS, 4),
                     "traffic": recorded_traffic(dom, "batch"), "alg_bytes_per_run": kd["alg_bytes_per_run"],
                     "us_per_run": kd["us_per_run"], "launches_per_run": kd["launches_per_run"]},
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def bench_serve(args):
    """Serving: Poisson-arriving compress/decompress requests against the
    continuous-batching server and against a serial FIFO server (one slot,
    one request per launch), at rates relative to the serial capacity."""
    import numpy as np
    import torch
    from paper_2201_13020_amd import serve, synth

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    bases = {False: synth.batch_field(dict(dims=(256, 512, 512), dtype="float32", eb=1e-3, zero_regions=True,
                                           seed=13020 + 7100), dev).reshape(-1),
             True: synth.batch_field(dict(dims=(128, 512, 512), dtype="float64", eb=1e-3, zero_regions=True,
                                          seed=13020 + 7101), dev).reshape(-1)}
    torch.cuda.synchronize()
    _log(f"generated base fields in {time.perf_counter() - t0:.1f} s")
    n_req = args.serve_requests
    warm = synth.serve_trace(256, 0.0, seed=1)
    warm["kind"][:] = 0
    policies = {"continuous_batching": dict(slots=args.serve_slots, max_batch=args.serve_max_batch),
                "serial_fifo": dict(slots=1, max_batch=1)}
    levels = [0.25, 0.5, 0.75, 0.9, 1.0, 1.1, 1.25]
    # the batching server goes on past the serial capacity, to its own knee
    extra = {"continuous_batching": [2.0, 3.0, 4.0, 5.0, 6.0], "serial_fifo": []}
    out = {}
    capacity = {}
    for name in ("serial_fifo", "continuous_batching"):
        pol = policies[name]
        with serve.Server(hbm_budget=args.serve_budget_gib << 30, block=BLOCK, **pol) as srv:
            _, pool = serve.replay(srv, warm, bases)
            sat = synth.serve_trace(n_req, 0.0, seed=2)
            done, pool = serve.replay(srv, sat, bases, warm_items=pool)
            s = serve.summarize(done)
            span = (max(c["t_done"] for c in done) - min(c["t_arrival"] for c in done)) / 1e9
            capacity[name] = dict(req_per_s=round(len(done) / span, 1), **s)
            _log(f"{name} saturated: {capacity[name]}")
            if name == "serial_fifo":
                base_rate = len(done) / span
            rows = {}
            for lv in levels + extra[name]:
                tr = synth.serve_trace(n_req, lv * base_rate, seed=100 + int(lv * 100))
                done, pool = serve.replay(srv, tr, bases, warm_items=pool)
                rows[str(lv)] = serve.summarize(done)
                _log(f"{name} load {lv}: {rows[str(lv)]}")
            st = srv.stats()
            out[name] = dict(levels=rows, arena_peak_GiB=round(st["arena_peak"] / 2**30, 2),
                             groups_launched=st["groups_launched"])
    cb, sf = out["continuous_batching"]["levels"], out["serial_fifo"]["levels"]
    result = {
        "metric": "compress & decompress GB/s (uncompressed) and % of HBM peak; ratio",
        "value": capacity["continuous_batching"]["GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": n_req,
        "warmup": 256,
        "ms_per_step": round(1e3 / capacity["continuous_batching"]["req_per_s"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, 60% compress / 40% decompress of resident streams, "
                               "sizes lognormal 64 KiB-256 MiB (median 4 MiB), 20% float64, REL 1e-3, block 128, "
                               f"HBM budget {args.serve_budget_gib} GiB; value = saturated continuous-batching "
                               "throughput (all requests queued at once)",
                   "requests_per_level": n_req, "slots": args.serve_slots, "max_batch": args.serve_max_batch,
                   "parallelism": "single GPU"},
        "detail": {
            "capacity": capacity,
            "load_levels_x_serial_capacity": levels,
            "extra_levels_batching_only": extra["continuous_batching"],
            "serial_capacity_req_per_s": capacity["serial_fifo"]["req_per_s"],
            "policies": out,
            "p99_ms_ratio_serial_over_batching": {lv: round(sf[lv]["p99_ms"] / cb[lv]["p99_ms"], 2) for lv in sf},
        },
    }
    print(json.dumps(result), flush=True)



def bench_shard(args):
    """The 2^28 float64 state vector as G contiguous block-range shards on one
    GPU (the single-GPU share of a G-GPU run, each shard in turn): the shards'
    ranges, each shard's compression with the whole field's bound, and the
    stitch of the shard streams into the field's stream, against the plain
    whole-field compression; the stitched stream is checked equal to it."""
    import numpy as np
    import torch
    from paper_2201_13020_amd import synth, szx

    dev = torch.device("cuda:0")
    x_np = synth.make("state")
    x = torch.from_numpy(x_np).to(dev)
    n, block, eb = x.numel(), BLOCK, 1e-3
    nbytes = n * 8
    field = szx.make_params(torch.float64, (n,), eb, "rel", block)
    whole, wsize = szx.compress(x, eb, "rel", block)
    torch.cuda.synchronize()
    wn = int(wsize.cpu().view(torch.int64).item())
    ws_whole = torch.empty(szx.workspace_size(torch.float64, (n,), eb, "rel", block), dtype=torch.uint8, device=dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(3, args.steps // 4)
    t_whole = timed(lambda: szx.compress(x, eb, "rel", block, out=whole, out_size=wsize, ws=ws_whole), reps)
    rows = {}
    for G in [int(g) for g in args.shards.split(",")]:
        nblk = -(-n // block)
        edges = [0] + sorted({8 * round(i * nblk / G / 8) for i in range(1, G)} - {0, nblk}) + [nblk]
        bounds = list(zip(edges[:-1], edges[1:]))
        parts = [x[k0 * block:min(n, k1 * block)] for k0, k1 in bounds]
        sps = [szx.shard_params(field, k0, k1) for k0, k1 in bounds]
        ranges = torch.empty(2 * G, dtype=torch.float64, device=dev)
        wss = [torch.empty(int(szx.lib().sz_workspace_size(sp_byref(sp))), dtype=torch.uint8, device=dev) for sp in sps]
        outs = [torch.empty(int(szx.lib().sz_compress_bound(sp_byref(sp))), dtype=torch.uint8, device=dev)
                for sp in sps]
        sizes = [torch.zeros(1, dtype=torch.uint64, device=dev) for _ in sps]
        st_out = torch.empty_like(whole)
        st_size = torch.zeros(1, dtype=torch.uint64, device=dev)

        def ranges_all():
            for i, xs in enumerate(parts):
                szx.field_range(xs, block, ws=wss[i], out=ranges[2 * i:2 * i + 2])

        def compress_all():
            for i, ((k0, k1), xs) in enumerate(zip(bounds, parts)):
                szx.compress_shard(field, k0, k1, xs, ranges, out=outs[i], out_size=sizes[i], ws=wss[i])

        def stitch_all():
            szx.stitch(field, outs, out=st_out, out_size=st_size)

        t_r = timed(ranges_all, reps)
        t_c = timed(compress_all, reps)
        t_s = timed(stitch_all, reps)
        torch.cuda.synchronize()
        sn = int(st_size.cpu().view(torch.int64).item())
        assert sn == wn and torch.equal(st_out[:sn], whole[:wn]), f"G={G}: stitched stream differs"
        rows[str(G)] = {"range_ms": round(t_r, 4), "compress_shards_ms": round(t_c, 4), "stitch_ms": round(t_s, 4),
                        "per_shard_compress_ms": round(t_c / G, 4),
                        "stitch_GBps_of_stream": round(2 * sn / t_s / 1e6, 1),
                        "total_GBps_uncompressed": round(nbytes / (t_r + t_c + t_s) / 1e6, 1)}
        _log(f"shard G={G}: {rows[str(G)]}")
    result = {
        "metric": "compress GB/s (uncompressed) of a field as shards + stitch, one GPU",
        "value": rows[max(rows, key=int)]["total_GBps_uncompressed"],
        "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 1, "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2^28 float64 state vector, REL 1e-3, block 128, in G contiguous block-range shards "
                               "compressed one after another on one GPU, then stitched; value: the largest G",
                   "parallelism": "single GPU"},
        "detail": {"whole_field_compress_ms": round(t_whole, 4),
                   "whole_field_GBps": round(nbytes / t_whole / 1e6, 1), "ratio": round(nbytes / wn, 4),
                   "shards": rows},
    }
    print(json.dumps(result), flush=True)


def sp_byref(sp):
    import ctypes
    return ctypes.byref(sp)


def _mount_of(path):
    """(mount point, filesystem type) holding path, from /proc/mounts."""
    best = ("", "unknown")
    try:
        real = os.path.realpath(path)
        for line in open("/proc/mounts"):
            parts = line.split()
            if len(parts) >= 3 and (real == parts[1] or real.startswith(parts[1].rstrip("/") + "/")):
                if len(parts[1]) > len(best[0]):
                    best = (parts[1], parts[2])
    except OSError:
        pass
    return best


def bench_io(args):
    """Dumping and loading a field through files, with and without
    compression: the single-node counterpart of the paper's dumping/loading
    breakdown (Sec. VI). Dump = compress on the GPU + write the stream to a
    file; load = read the file into device memory + decompress. Raw = the
    uncompressed field written and read the same way. Each leg is timed on its
    own (device synchronised around it), the median of --steps repetitions.
    Writes go through the page cache, and a second set flushes every file to
    storage (fsync); reads come back from the page cache (the files were just
    written and nothing evicts them)."""
    import shutil
    import statistics
    import tempfile
    import numpy as np
    import torch
    from paper_2201_13020_amd import synth, szx

    field = FIELDS["turbulence"]
    shape = field["shape"]
    x_np = synth.make("turbulence")
    x = torch.from_numpy(x_np).cuda()
    nbytes = x.numel() * x.element_size()
    own_dir = args.io_dir is None
    d = tempfile.mkdtemp(prefix="szx_io_") if own_dir else args.io_dir
    mount, fstype = _mount_of(d)
    reps = max(1, min(args.steps, 5))
    _log(f"io: {nbytes / 1e6:.0f} MB field, files under {d} ({fstype} at {mount}), {reps} repetitions")

    def timed(fn):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    rows = {}
    try:
        raw_path = os.path.join(d, "raw.bin")
        for durable in (False, True):
            tag = "fsync" if durable else "page_cache"
            raw_w = timed(lambda: szx.file_write(raw_path, x, durable=durable))
            back = torch.empty_like(x)
            raw_r = timed(lambda: szx.file_read(raw_path, out=back))
            assert torch.equal(back, x)
            rows[tag] = {"raw": {"write_ms": round(raw_w * 1e3, 3), "read_ms": round(raw_r * 1e3, 3),
                                 "dump_GBps": round(nbytes / raw_w / 1e9, 2),
                                 "load_GBps": round(nbytes / raw_r / 1e9, 2)}}
            for eb in field["bounds"]:
                out, size = szx.compress(x, eb, "rel", BLOCK)
                torch.cuda.synchronize()
                n = int(size.cpu().view(torch.int64).item())
                ws = torch.empty(szx.workspace_size(torch.float32, shape, eb, "rel", BLOCK), dtype=torch.uint8,
                                 device="cuda")
                t_c = timed(lambda: szx.compress(x, eb, "rel", BLOCK, out=out, out_size=size, ws=ws))
                path = os.path.join(d, f"s{eb}.szx")
                t_w = timed(lambda: szx.file_write(path, out, nbytes=n, durable=durable))
                sbuf = torch.empty(n, dtype=torch.uint8, device="cuda")
                t_r = timed(lambda: szx.file_read(path, out=sbuf))
                params = dict(dtype=torch.float32, dims=shape, block=BLOCK)
                y, st = szx.decompress(sbuf, n, params)
                t_d = timed(lambda: szx.decompress(sbuf, n, params, out=y, status=st, ws=ws))
                assert int(st.cpu().view(torch.int32).item()) == 0 and torch.equal(sbuf, out[:n])
                err = float((y.reshape(-1).double() - x.reshape(-1).double()).abs().max())
                dump, load = t_c + t_w, t_r + t_d
                rows[tag][str(eb)] = {
                    "ratio": round(nbytes / n, 4), "compress_ms": round(t_c * 1e3, 3), "write_ms": round(t_w * 1e3, 3),
                    "read_ms": round(t_r * 1e3, 3), "decompress_ms": round(t_d * 1e3, 3),
                    "dump_GBps": round(nbytes / dump / 1e9, 2), "load_GBps": round(nbytes / load / 1e9, 2),
                    "dump_speedup_vs_raw": round(raw_w / dump, 2), "load_speedup_vs_raw": round(raw_r / load, 2),
                    "max_abs_error": err}
                _log(f"io {tag} eb={eb}: dump {dump * 1e3:.2f} ms (raw {raw_w * 1e3:.2f}), "
                     f"load {load * 1e3:.2f} ms (raw {raw_r * 1e3:.2f})")
    finally:
        if own_dir:
            shutil.rmtree(d, ignore_errors=True)
    mid = rows["fsync"][str(1e-3)]
    result = {
        "metric": "dump + load GB/s of uncompressed bytes (compress + write, read + decompress)",
        "value": round(2 * nbytes / ((mid["compress_ms"] + mid["write_ms"] + mid["read_ms"] + mid["decompress_ms"]) / 1e3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": 0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"100x500x500 float32 turbulence field dumped to and loaded from files on {fstype}, "
                               f"REL 1e-2/1e-3/1e-4, block 128; value: REL 1e-3 with fsync",
                   "filesystem": fstype, "parallelism": "single GPU"},
        "detail": rows,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
