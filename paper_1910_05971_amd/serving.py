"""Continuous-batching server (C ABI fastsv_server_*) and open-loop drivers.

``Server`` wraps one device pool.  Requests are host CSR graphs; each
``step()`` admits queued graphs that fit, runs one iteration of the method for
every running graph and delivers the ones that converged in it (their labels
land in the numpy buffer handed back by ``poll()``).

``run_open_loop`` replays a request trace with scheduled arrival times against
the server; ``run_plain`` replays it against the one-graph-per-call path
(FIFO, ``cc_csr`` per request).  Both report per-request latency from the
scheduled arrival to the moment the labels are on the host.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import binding as B


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("dense_steps", ctypes.c_int64), ("sparse_steps", ctypes.c_int64),
                ("cancelled", ctypes.c_int64)]


def _bind(lib):
    if getattr(lib, "_server_bound", False):
        return lib
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.fastsv_server_pool_bytes.restype = ctypes.c_size_t
    lib.fastsv_server_pool_bytes.argtypes = [i32, i64, i32]
    lib.fastsv_server_create.restype = ctypes.c_int
    lib.fastsv_server_create.argtypes = [vp, i32, i64, i32, vp, ctypes.POINTER(B.Opts), ctypes.POINTER(vp)]
    lib.fastsv_server_destroy.restype = None
    lib.fastsv_server_destroy.argtypes = [vp]
    lib.fastsv_server_submit.restype = ctypes.c_int
    lib.fastsv_server_submit.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.POINTER(u64)]
    lib.fastsv_server_submit_mapped.restype = ctypes.c_int
    lib.fastsv_server_submit_mapped.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.POINTER(u64)]
    lib.fastsv_server_submit_batch.restype = ctypes.c_int
    lib.fastsv_server_submit_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, i32, ctypes.POINTER(i32)]
    lib.fastsv_server_step.restype = ctypes.c_int
    lib.fastsv_server_step.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.fastsv_server_poll.restype = ctypes.c_int
    lib.fastsv_server_poll.argtypes = [vp, ctypes.POINTER(u64), i32, ctypes.POINTER(i32)]
    lib.fastsv_server_cancel.restype = ctypes.c_int
    lib.fastsv_server_cancel.argtypes = [vp, u64]
    lib.fastsv_server_get_stats.restype = ctypes.c_int
    lib.fastsv_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib._server_bound = True
    return lib


def pool_bytes(max_vertices, max_entries, max_slots):
    return int(_bind(B.load_library()).fastsv_server_pool_bytes(max_vertices, max_entries, max_slots))


class Server:
    def __init__(self, max_vertices: int, max_entries: int, max_slots: int, device: int = 0,
                 frontier_tau: float | None = None, validate: bool = True, admit_mb: int | None = None):
        self.lib = _bind(B.load_library())
        self.device = device
        torch.cuda.set_device(device)
        self.stream = torch.cuda.current_stream(device)
        opts = B.make_opts(frontier_tau=frontier_tau, validate=validate)
        if admit_mb is not None:
            opts.admit_mb = int(admit_mb)
        h = ctypes.c_void_p()
        st = self.lib.fastsv_server_create(B.context(device), int(max_vertices), int(max_entries), int(max_slots),
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(opts),
                                           ctypes.byref(h))
        if st != B.FASTSV_OK:
            raise B.FastSVError(st, "fastsv_server_create")
        self.h = h
        self.pending = {}  # ticket -> (labels, iters, rp, col) kept alive until done
        self._done = (ctypes.c_uint64 * 4096)()  # poll buffer, reused
        self._nd = ctypes.c_int32()
        self._r, self._q = ctypes.c_int32(), ctypes.c_int32()

    def submit(self, row_ptr: np.ndarray, col: np.ndarray, mapped: bool = False) -> int:
        """mapped=True: row_ptr and col are page-locked arrays from pin_graphs
        (fastsv_server_submit_mapped)."""
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        n = rp.shape[0] - 1
        labels = np.empty(max(n, 1), dtype=np.int32)
        iters = np.zeros(1, dtype=np.int32)
        t = ctypes.c_uint64()
        fn = self.lib.fastsv_server_submit_mapped if mapped else self.lib.fastsv_server_submit
        st = fn(self.h, n, int(cl.shape[0]), ctypes.c_void_p(rp.ctypes.data), ctypes.c_void_p(cl.ctypes.data),
                ctypes.c_void_p(labels.ctypes.data), ctypes.c_void_p(iters.ctypes.data), ctypes.byref(t))
        if st != B.FASTSV_OK:
            raise B.FastSVError(st, "fastsv_server_submit")
        # the server reads rp/col at admission: keep them alive until done
        self.pending[t.value] = (labels[:n], iters, rp, cl)
        return t.value

    def submit_many(self, graphs, mapped: bool = False) -> list[int]:
        """Submit many requests in one library call (fastsv_server_submit_batch);
        graphs are objects with row_ptr and col (int32, contiguous).  Returns
        the tickets in order."""
        k = len(graphs)
        if k == 0:
            return []
        rps = [np.ascontiguousarray(g.row_ptr, dtype=np.int32) for g in graphs]
        cols = [np.ascontiguousarray(g.col, dtype=np.int32) for g in graphs]
        n = np.array([r.shape[0] - 1 for r in rps], dtype=np.int32)
        nnz = np.array([c.shape[0] for c in cols], dtype=np.int64)
        labels = np.empty(int(np.maximum(n, 1).sum()), dtype=np.int32)
        lab_off = np.concatenate([[0], np.cumsum(np.maximum(n, 1))[:-1]]).astype(np.int64)
        iters = np.zeros(k, dtype=np.int32)
        rp_p = np.array([r.ctypes.data for r in rps], dtype=np.uint64)
        col_p = np.array([c.ctypes.data for c in cols], dtype=np.uint64)
        lab_p = (labels.ctypes.data + 4 * lab_off).astype(np.uint64)
        tickets = np.zeros(k, dtype=np.uint64)
        acc = ctypes.c_int32()
        st = self.lib.fastsv_server_submit_batch(
            self.h, k, ctypes.c_void_p(n.ctypes.data), ctypes.c_void_p(nnz.ctypes.data),
            ctypes.c_void_p(rp_p.ctypes.data), ctypes.c_void_p(col_p.ctypes.data), ctypes.c_void_p(lab_p.ctypes.data),
            ctypes.c_void_p(iters.ctypes.data), ctypes.c_void_p(tickets.ctypes.data), int(bool(mapped)),
            ctypes.byref(acc))
        # one shared record per call; a ticket maps to (record, index), and the
        # labels view is cut when the ticket is polled
        rec = (labels, lab_off.tolist(), n.tolist(), iters, rps, cols)
        tl = tickets.tolist()
        self.pending.update(zip(tl[:acc.value], ((rec, i) for i in range(acc.value))))
        if st != B.FASTSV_OK:
            raise B.FastSVError(st, "fastsv_server_submit_batch")
        return tl

    def step(self):
        r, q = self._r, self._q
        st = self.lib.fastsv_server_step(self.h, ctypes.byref(r), ctypes.byref(q))
        if st != B.FASTSV_OK:
            raise B.FastSVError(st, "fastsv_server_step")
        return r.value, q.value

    def cancel(self, ticket: int) -> int:
        """fastsv_server_cancel: FASTSV_OK, FASTSV_EBUSY (admission copies
        still in flight: try again after a step) or FASTSV_EINVAL (unknown or
        already delivered).  A cancelled ticket is never reported by poll()."""
        st = self.lib.fastsv_server_cancel(self.h, ctypes.c_uint64(ticket))
        if st == B.FASTSV_OK:
            self.pending.pop(ticket, None)
        return st

    def poll(self):
        buf, k = self._done, self._nd
        cap = len(buf)
        out = []
        while True:
            st = self.lib.fastsv_server_poll(self.h, buf, cap, ctypes.byref(k))
            if st != B.FASTSV_OK:
                raise B.FastSVError(st, "fastsv_server_poll")
            if k.value == 0:
                return out
            for t in buf[:k.value]:
                p = self.pending.pop(t)
                if len(p) == 2:  # from submit_many: (shared record, index)
                    (labels, off, n, iters, _, _), i = p
                    out.append((t, labels[off[i]:off[i] + n[i]], int(iters[i])))
                else:
                    lab, its, _, _ = p
                    out.append((t, lab, int(its[0])))
            if k.value < cap:
                return out

    def stats(self) -> ServerStats:
        s = ServerStats()
        self.lib.fastsv_server_get_stats(self.h, ctypes.byref(s))
        return s

    def close(self):
        if self.h:
            self.lib.fastsv_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_open_loop(server: Server, graphs, arrivals, on_done=None, idle_sleep=0.0, mapped=False):
    """Replay requests graphs[i] (objects with row_ptr/col) arriving at
    arrivals[i] seconds after the start.  Returns (latency seconds per request,
    makespan seconds, iterations per request)."""
    order = np.argsort(arrivals, kind="stable")
    lat = np.full(len(graphs), np.nan)
    iters = np.zeros(len(graphs), dtype=np.int64)
    ticket_of = {}
    t0 = time.perf_counter()
    nxt = 0
    outstanding = 0
    while nxt < len(order) or outstanding:
        now = time.perf_counter() - t0
        arrived = []
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            arrived.append(int(order[nxt]))
            nxt += 1
        if len(arrived) == 1:
            i = arrived[0]
            ticket_of[server.submit(graphs[i].row_ptr, graphs[i].col, mapped=mapped)] = i
        elif arrived:
            for i, t in zip(arrived, server.submit_many([graphs[i] for i in arrived], mapped=mapped)):
                ticket_of[t] = i
        outstanding += len(arrived)
        if outstanding:
            resident, queued = server.step()
            # poll only when some request has left the server
            if resident + queued >= outstanding:
                continue
            for t, lab, its in server.poll():
                i = ticket_of.pop(t)
                lat[i] = time.perf_counter() - t0 - arrivals[i]
                iters[i] = its
                outstanding -= 1
                if on_done:
                    on_done(i, lab, its)
        elif nxt < len(order):
            wait = arrivals[order[nxt]] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.001) if idle_sleep == 0.0 else idle_sleep)
    return lat, time.perf_counter() - t0, iters


def run_plain(graphs, arrivals, device=0, on_done=None):
    """FIFO, one request at a time through fastsv_cc_csr (host -> device copy,
    solve, labels back to the host)."""
    order = np.argsort(arrivals, kind="stable")
    lat = np.full(len(graphs), np.nan)
    iters = np.zeros(len(graphs), dtype=np.int64)
    dev = torch.device("cuda", device)
    t0 = time.perf_counter()
    for i in order:
        i = int(i)
        wait = arrivals[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        g = graphs[i]
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(dev)
        col = torch.from_numpy(np.ascontiguousarray(g.col)).to(dev)
        labels, st = B.cc_csr(rp, col)
        lab = labels.cpu().numpy()
        lat[i] = time.perf_counter() - t0 - arrivals[i]
        iters[i] = st.iterations
        if on_done:
            on_done(i, lab, st.iterations)
    return lat, time.perf_counter() - t0, iters


def pin_graphs(graphs):
    """Copy each distinct graph's CSR into page-locked host memory (so the
    host-to-device copies of both paths are plain DMA); returns the list with
    the same sharing as the input."""
    from .graphgen import Graph
    done = {}
    out = []
    for g in graphs:
        key = id(g)
        if key not in done:
            rp = torch.empty(g.row_ptr.shape[0], dtype=torch.int32, pin_memory=True).numpy()
            col = torch.empty(max(g.col.shape[0], 1), dtype=torch.int32, pin_memory=True).numpy()[:g.col.shape[0]]
            rp[:] = g.row_ptr
            col[:] = g.col
            done[key] = Graph(g.name, g.n, rp, col, g.m_eff)
        out.append(done[key])
    return out
