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
                ("t_done", ctypes.c_uint64), ("group_size", ctypes.c_uint32), ("slot", ctypes.c_uint32)]


class SzServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("arena_bytes", "arena_in_use", "arena_peak", "queued",
                                               "in_flight_groups", "groups_launched", "completed",
                                               "items_resident")]


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


def replay(server, trace, bases, eb=1e-3, warm_items=(), keep_items=512, rng_seed=0, timeout_s=600.0):
    """Submit the requests of `trace` (see synth.serve_trace) at their arrival
    times and wait for all completions.

    bases: {False: float32 device field, True: float64 device field}; a
    compression reads a 16-byte-aligned slice of the base of its type.
    Decompressions write into the arena and their outputs are released as
    they complete. warm_items: resident items to start the pick pool with;
    the pool keeps at most keep_items items (the oldest are released).
    Returns (completions in request order, pool items still resident)."""
    L = _lib()
    n = len(trace["t"])
    t = trace["t"]
    pool = list(warm_items)
    pending = {}
    done = []
    # parameters built before the clock starts
    plan = []
    for i in range(n):
        if trace["kind"][i] == SZ_REQ_COMPRESS:
            f64 = bool(trace["f64"][i])
            base = bases[f64]
            w = 8 if f64 else 4
            cnt = max(1, int(trace["nbytes"][i]) // w)
            room = base.numel() - cnt
            off = int(trace["pos"][i] * max(room, 0)) // 4 * 4
            p = szx.make_params(base.dtype, (cnt,), eb, "rel", server.block)
            plan.append((base, off * w, p))
        else:
            plan.append(None)

    def collect(wait_us=0):
        for c in server.poll(wait_us):
            kind = pending.pop(c["request"])
            done.append(c)
            if c["status"] != 0:
                continue
            if kind == SZ_REQ_COMPRESS:
                pool.append(c["item"])
                if len(pool) > keep_items:
                    server.release(pool.pop(0))
            elif c["out_item"]:
                server.release(c["out_item"])

    start = server.clock() + 2_000_000  # 2 ms from now
    rid = ctypes.c_uint64()
    for i in range(n):
        due = start + int(t[i] * 1e9)
        while server.clock() < due:
            collect()
        if plan[i] is not None:
            base, boff, p = plan[i]
            rc = L.sz_server_submit_compress(server._h, ctypes.byref(p), base.data_ptr() + boff, due, ctypes.byref(rid))
            _check(rc, "submit compress")
            pending[rid.value] = SZ_REQ_COMPRESS
        else:
            if not pool:
                continue
            item = pool[int(trace["pos"][i] * len(pool)) % len(pool)]
            rc = L.sz_server_submit_decompress(server._h, item, None, 0, due, ctypes.byref(rid))
            _check(rc, "submit decompress")
            pending[rid.value] = SZ_REQ_DECOMPRESS
    t_end = time.time() + timeout_s
    while pending and time.time() < t_end:
        collect(10_000)
    if pending:
        raise TimeoutError(f"{len(pending)} requests still pending")
    done.sort(key=lambda c: c["request"])
    return done, pool


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
