"""Autotuner of the launch geometry of the encode pass.

A single-knob tuner: the knob is the number of persistent workgroups of the
encode kernel, per element type. It never changes the output bytes; it only
trades the cost of idle workgroups against the latency hidden by more of
them. The best value depends on the device and on how much data a launch
covers, so it is measured per (device, block size, element type, size class)
and cached in a JSON file ($SZX_TUNE_CACHE, default ~/.cache/szx/tune.json).
apply_cache loads the entries of one device and block size into the
library's process-wide table (per element type and size class), which
sz_compress and new batches consult. The other launch parameters (tile bytes
of the passes) are compile-time constants of the kernels.
"""
import json
import os

import torch

from . import szx

MULTIPLIERS = (1, 2, 3, 4, 6, 8, 12, 16)


def cache_path():
    return os.environ.get("SZX_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "szx", "tune.json"))


def device_key(device=None):
    """"<arch>|cu<compute units>" of a torch device (index or None for the
    current one); a string is taken as a key already."""
    if isinstance(device, str):
        return device
    p = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}|cu{p.multi_processor_count}"


def _compute_units(dev_key):
    return int(dev_key.rsplit("|cu", 1)[1])


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(entries):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(dev, block, dtype, cls):
    return f"{dev}|b{block}|{dtype}|c{cls}"


def apply_cache(device=None, block=128):
    """Load the cached geometries of this device tuned at block size `block`
    into the library table. Returns the number of entries applied."""
    dev = device_key(device)
    want = f"b{int(block)}"
    n = 0
    for k, v in _load().items():
        parts = k.split("|")
        if len(parts) != 5 or "|".join(parts[:2]) != dev or parts[2] != want:
            continue
        szx.set_geometry(parts[3], int(parts[4][1:]), int(v["encode_wgs"]))
        n += 1
    return n


def _time(fn, reps):
    s = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune_batch(batch, bytes_per_dtype, block=128, reps=5, multipliers=MULTIPLIERS, store=True,
               timer=None, device=None):
    """Time batch.run() over the candidate encode geometries of each element
    type present (bytes_per_dtype: {"float32": bytes, "float64": bytes}), keep
    the fastest in the batch, the library table and the cache. `block` is the
    block size of the batch's fields (part of the cache key); `timer(fn,
    reps)` returns the time of fn in ms (default: the median of reps runs
    between device events); `device` is a device index or key. Returns
    {dtype: (encode_wgs, ms, {candidate: ms})}."""
    dev = device_key(device)
    ncu = _compute_units(dev)
    timer = _time if timer is None else timer
    entries = _load() if store else {}
    result = {}
    batch.run()  # warm
    for dtype, nbytes in bytes_per_dtype.items():
        if nbytes <= 0:
            continue
        times = {}
        for m in multipliers:
            batch.set_geometry(m * ncu, dtype)
            times[m * ncu] = timer(batch.run, reps)
        best = min(times, key=times.get)
        batch.set_geometry(best, dtype)
        cls = szx.size_class(nbytes)
        szx.set_geometry(dtype, cls, best)
        entries[_key(dev, block, dtype, cls)] = dict(encode_wgs=best, ms=times[best], bytes=int(nbytes))
        result[dtype] = (best, times[best], times)
    if store:
        _store(entries)
    return result
