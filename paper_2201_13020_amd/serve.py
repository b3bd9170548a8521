"""Python binding of the serving runtime in include/szx_server.h, and the
load driver that replays a request trace against it.

The runtime is native (libszx.so): admission, grouping, launches and
completion all happen in its threads. This module marshals arguments,
submits requests at their arrival times and collects completions.
"""
import ctypes
import time

import numpy as np
import torch

from . import szx

SZ_REQ_COMPRESS, SZ_REQ_DECOMPRESS = 0, 1


class SzServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("block_size", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class SzCompletion(ctypes.Structure):
    _fields_ = [("request", ctypes.c_uint64), ("kind", ctypes.c_uint32), ("status", ctypes.c_uint32),
                ("item", ctypes.c_uint64), ("out_item", ctypes.c_uint64), ("bytes_in", ctypes.c_uint64),
                ("stream_bytes", ctypes.c_uint64), ("t_arrival", ctypes.c_uint64), ("t_admit", ctypes.c_uint64),
                ("t_done", ctypes.c_uint64), ("group_size", ctypes.c_uint32), ("slot", ctypes.c_uint32),
                ("t_dev_begin", ctypes.c_uint64), ("t_dev_end", ctypes.c_uint64)]


class SzTraceReq(ctypes.Structure):
    _fields_ = [("t_arrival", ctypes.c_uint64), ("kind", ctypes.c_uint32), ("pick", ctypes.c_uint32),
                ("params", szx.SzParams), ("d_in", ctypes.c_void_p)]


class SzServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("arena_bytes", "arena_in_use", "arena_peak", "queued",
                                               "in_flight_groups", "groups_launched", "completed",
                                               "items_resident", "peak_in_flight_groups")]


_bound = False


def _lib():
    global _bound
    L = szx.lib()
    if not _bound:
        vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        L.sz_server_create.argtypes = [ctypes.POINTER(SzServerConfig), ctypes.POINTER(vp)]
        L.sz_server_create.restype = ctypes.c_int
        L.sz_server_destroy.argtypes = [vp]
        L.sz_server_destroy.restype = None
        L.sz_server_clock.argtypes = [vp]
        L.sz_server_clock.restype = u64
        L.sz_server_submit_compress.argtypes = [vp, ctypes.POINTER(szx.SzParams), vp, u64, ctypes.POINTER(u64)]
        L.sz_server_submit_compress.restype = ctypes.c_int
        L.sz_server_submit_decompress.argtypes = [vp, u64, vp, u64, u64, ctypes.POINTER(u64)]
        L.sz_server_submit_decompress.restype = ctypes.c_int
        L.sz_server_poll.argtypes = [vp, ctypes.POINTER(SzCompletion), u32, u32]
        L.sz_server_poll.restype = u32
        L.sz_server_item_info.argtypes = [vp, u64, ctypes.POINTER(szx.SzParams), ctypes.POINTER(u64),
                                          ctypes.POINTER(vp)]
        L.sz_server_item_info.restype = ctypes.c_int
        L.sz_server_copy_item.argtypes = [vp, u64, vp, u64, vp]
        L.sz_server_copy_item.restype = ctypes.c_int
        L.sz_server_release.argtypes = [vp, u64]
        L.sz_server_release.restype = ctypes.c_int
        L.sz_server_get_stats.argtypes = [vp, ctypes.POINTER(SzServerStats)]
        L.sz_server_get_stats.restype = ctypes.c_int
        L.sz_server_replay.argtypes = [vp, ctypes.POINTER(SzTraceReq), u32, ctypes.POINTER(u64), u32, u32, u32,
                                       ctypes.POINTER(SzCompletion), ctypes.POINTER(u64), ctypes.POINTER(u32)]
        L.sz_server_replay.restype = ctypes.c_int
        _bound = True
    return L


def _check(rc, what):
    if rc != 0:
        raise szx.SzError(rc, f"{what}: {szx.lib().sz_last_error().decode()}")


class Server:
    """A serving runtime on one device. Inputs passed to submit_compress and
    outputs passed to submit_decompress are kept referenced until their
    completion has been polled."""

    def __init__(self, hbm_budget=64 << 30, slots=4, max_batch=64, block=128, device=0):
        c = SzServerConfig(device=device, hbm_budget=int(hbm_budget), slots=slots, max_batch=max_batch,
                           block_size=block, reserved=0)
        h = ctypes.c_void_p()
        _check(_lib().sz_server_create(ctypes.byref(c), ctypes.byref(h)), "sz_server_create")
        self._h = h
        self.block = block
        self._keep = {}
        self._buf = (SzCompletion * 1024)()

    def close(self):
        if self._h:
            _lib().sz_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self):
        return int(_lib().sz_server_clock(self._h))

    def submit_compress(self, x, eb, mode="rel", dims=None, t_arrival=0, params=None):
        p = params if params is not None else szx.make_params(x.dtype, dims or (tuple(x.shape) or (1,)), eb, mode,
                                                              self.block)
        rid = ctypes.c_uint64()
        _check(_lib().sz_server_submit_compress(self._h, ctypes.byref(p), x.data_ptr(), int(t_arrival),
                                                ctypes.byref(rid)), "sz_server_submit_compress")
        self._keep[rid.value] = x
        return rid.value

    def submit_decompress(self, item, out=None, t_arrival=0):
        rid = ctypes.c_uint64()
        ptr = out.data_ptr() if out is not None else None
        cap = out.numel() * out.element_size() if out is not None else 0
        _check(_lib().sz_server_submit_decompress(self._h, int(item), ptr, cap, int(t_arrival), ctypes.byref(rid)),
               "sz_server_submit_decompress")
        if out is not None:
            self._keep[rid.value] = out
        return rid.value

    def poll(self, wait_us=0):
        """Completions as a list of dicts (at most 1024 per call)."""
        k = _lib().sz_server_poll(self._h, self._buf, len(self._buf), int(wait_us))
        out = []
        for i in range(k):
            c = self._buf[i]
            self._keep.pop(c.request, None)
            out.append({f: getattr(c, f) for f, _ in SzCompletion._fields_})
        return out

    def item_info(self, item):
        p = szx.SzParams()
        nb = ctypes.c_uint64()
        ptr = ctypes.c_void_p()
        _check(_lib().sz_server_item_info(self._h, int(item), ctypes.byref(p), ctypes.byref(nb), ctypes.byref(ptr)),
               "sz_server_item_info")
        return szx.params_dict(p), int(nb.value), ptr.value

    def read_item(self, item):
        """A device uint8 tensor with a copy of the item's bytes."""
        _, nb, _ = self.item_info(item)
        dst = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
        _check(_lib().sz_server_copy_item(self._h, int(item), dst.data_ptr(), dst.numel(),
                                          szx._stream_handle(None)), "sz_server_copy_item")
        return dst[:nb]

    def release(self, item):
        _check(_lib().sz_server_release(self._h, int(item)), "sz_server_release")

    def stats(self):
        s = SzServerStats()
        _check(_lib().sz_server_get_stats(self._h, ctypes.byref(s)), "sz_server_get_stats")
        return {f: int(getattr(s, f)) for f, _ in SzServerStats._fields_}


def replay(server, trace, bases, eb=1e-3, warm_items=(), keep_items=512, timeout_s=600.0):
    """Replay `trace` (see synth.serve_trace) through the server with the
    library's native load driver (sz_server_replay): requests are submitted
    at their arrival times, compressions read 16-byte-aligned slices of
    bases[f64] (a float32 and a float64 device field), decompressions pick
    resident items and write into the arena (released on completion).
    warm_items start the pick pool (at most keep_items kept). Returns
    (completions in request order, pool items still resident)."""
    n = len(trace["t"])
    reqs = (SzTraceReq * max(n, 1))()
    start = server.clock() + 2_000_000  # 2 ms from now, after this set-up
    for i in range(n):
        r = reqs[i]
        r.t_arrival = start + int(trace["t"][i] * 1e9)
        r.kind = int(trace["kind"][i])
        if r.kind == SZ_REQ_COMPRESS:
            f64 = bool(trace["f64"][i])
            base = bases[f64]
            w = 8 if f64 else 4
            cnt = max(1, int(trace["nbytes"][i]) // w)
            room = base.numel() - cnt
            off = int(trace["pos"][i] * max(room, 0)) // 4 * 4
            r.params = szx.make_params(base.dtype, (cnt,), eb, "rel", server.block)
            r.d_in = base.data_ptr() + off * w
        else:
            r.pick = int(trace["pos"][i] * (1 << 31))
    if start < server.clock():
        # set-up took longer than the margin: shift the whole trace
        lag = server.clock() - start + 1_000_000
        for i in range(n):
            reqs[i].t_arrival += lag
    warm = list(warm_items)
    cap = max(len(warm), keep_items)
    warm_arr = (ctypes.c_uint64 * max(len(warm), 1))(*warm)
    out = (SzCompletion * max(n, 1))()
    pool = (ctypes.c_uint64 * cap)()
    npool = ctypes.c_uint32()
    rc = _lib().sz_server_replay(server._h, reqs, n, warm_arr, len(warm), keep_items, int(timeout_s * 1000), out,
                                 pool, ctypes.byref(npool))
    _check(rc, "sz_server_replay")
    done = [{f: getattr(out[i], f) for f, _ in SzCompletion._fields_} for i in range(n)]
    return done, [int(pool[i]) for i in range(npool.value)]


def summarize(done):
    """p50/p99 latency (arrival to device completion) and throughput."""
    ok = [c for c in done if c["status"] == 0]
    lat = np.array([(c["t_done"] - c["t_arrival"]) / 1e6 for c in ok])
    t0 = min(c["t_arrival"] for c in ok)
    t1 = max(c["t_done"] for c in ok)
    nbytes = sum(c["bytes_in"] for c in ok)
    groups = np.array([c["group_size"] for c in ok])
    return {
        "requests": len(done), "failed": len(done) - len(ok),
        "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "mean_ms": round(float(lat.mean()), 4),
        "GBps": round(nbytes / ((t1 - t0) / 1e9) / 1e9, 2),
        "mean_group": round(float(groups.mean()), 2),
    }
