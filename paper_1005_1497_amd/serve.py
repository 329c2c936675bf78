"""Served form: continuous batching of exact circular convolutions.

Requests (f, g) of power-of-two lengths arrive at any time.  A scheduler thread

  1. admits queued requests, in arrival order, while device memory allows:
     each request takes one slot of its length from a buddy allocator over
     three equal device arenas (F, G, H), so one offset is valid in all three;
  2. copies the admitted requests' operands into their slots and launches them
     together as ONE conv_batched call (the fused forward / pointwise /
     inverse kernels) on the next of several HIP streams, so that batches
     admitted while others are still running overlap on the device;
  3. copies each result back, completes the request's future and frees its
     slot, which lets further requests in.

A request enters either by submit(f, g), which copies the operands into a pinned
staging buffer of the executor, or without that host copy: buffers(n) hands out
the staging buffer's operand rows, the caller writes f and g there in place and
passes the token to submit_staged().  Results are host arrays over the request's
pinned result row (no copy after the download); each stays valid while the
caller holds it.

Operands stay resident in the arenas from admission to completion.  Latency is
completion time minus arrival time on the host monotonic clock.

All arithmetic runs in the library's HIP kernels through conv_batched; this
module only schedules, allocates and copies.  The executor is pluggable so the
scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures
import threading
import time
from dataclasses import dataclass, field

import numpy as np


class BuddyAllocator:
    """Power-of-two buddy allocator over [0, 2^total_log2) elements.

    alloc(k) returns the offset of a free block of 2^k elements aligned to 2^k,
    or None when no such block is free; free(offset, k) returns it and merges
    buddies."""

    def __init__(self, total_log2: int, min_log2: int = 0):
        if min_log2 > total_log2:
            raise ValueError("min block larger than the arena")
        self.total_log2 = total_log2
        self.min_log2 = min_log2
        self.free_lists = {k: set() for k in range(min_log2, total_log2 + 1)}
        self.free_lists[total_log2].add(0)
        self.used = 0

    def alloc(self, k: int):
        k = max(k, self.min_log2)
        if k > self.total_log2:
            return None
        j = k
        while j <= self.total_log2 and not self.free_lists[j]:
            j += 1
        if j > self.total_log2:
            return None
        off = min(self.free_lists[j])
        self.free_lists[j].remove(off)
        while j > k:                 # split, keep the lower half
            j -= 1
            self.free_lists[j].add(off + (1 << j))
        self.used += 1 << k
        return off

    def free(self, off: int, k: int):
        k = max(k, self.min_log2)
        self.used -= 1 << k
        while k < self.total_log2:
            buddy = off ^ (1 << k)
            if buddy in self.free_lists[k]:
                self.free_lists[k].remove(buddy)
                off = min(off, buddy)
                k += 1
            else:
                break
        self.free_lists[k].add(off)

    @property
    def capacity(self) -> int:
        return 1 << self.total_log2


@dataclass
class Request:
    rid: int
    staged: object          # executor-specific staging of f, g and the output
    log2n: int
    arrival: float
    future: concurrent.futures.Future
    offset: int = -1
    done_time: float = 0.0
    out: np.ndarray = None
    cancelled: bool = False


@dataclass
class _Batch:
    reqs: list
    handle: object
    stream_id: int
    launched: float


# Statistics and the admission log keep the most recent entries only, so that
# a long-running server holds a bounded amount.
STATS_WINDOW = 1 << 20


@dataclass
class ServeStats:
    latencies: collections.deque = field(default_factory=lambda: collections.deque(maxlen=STATS_WINDOW))
    batch_sizes: collections.deque = field(default_factory=lambda: collections.deque(maxlen=STATS_WINDOW))
    peak_used: int = 0
    peak_inflight: int = 0
    completed: int = 0

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.array(self.latencies), q)) if self.latencies else float("nan")


@dataclass
class StagedToken:
    """A staging buffer handed out by ConvServer.buffers, not yet submitted."""
    staged: object
    log2n: int
    used: bool = False


class GpuExecutor:
    """Device side of the server: arenas, streams and conv_batched launches.

    Executor protocol (ConvServer calls only these): staging(n) -> a staging
    object for one request of length n; operand_views(staged) -> writable host
    arrays (f, g) inside it; prepare(f, g) -> a filled staging object;
    launch(requests, stream_id) -> handle; poll(handle) -> bool;
    results(handle) -> one host array per request; streams."""

    def __init__(self, m: int, capacity_log2: int, elem_bits: int = 64, streams: int = 2, device: int = 0,
                 root: int = 2, root_log2order: int | None = None):
        import torch
        import paper_1005_1497_amd as nt
        self.torch, self.nt = torch, nt
        self.m = m
        self.elem_bits = elem_bits
        self.dtype = torch.int64 if elem_bits == 64 else torch.int32
        self.np_dtype = np.uint64 if elem_bits == 64 else np.uint32
        self.dev = torch.device("cuda", device)
        n = 1 << capacity_log2
        # arenas: slots are written by uploads before any kernel reads them
        self.F = torch.empty(n, dtype=self.dtype, device=self.dev)
        self.G = torch.empty(n, dtype=self.dtype, device=self.dev)
        self.H = torch.empty(n, dtype=self.dtype, device=self.dev)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.wb = elem_bits // 8
        self.F_ptr, self.G_ptr, self.H_ptr = (np.uint64(t.data_ptr()) for t in (self.F, self.G, self.H))
        self.root = root
        self.rlo = root_log2order if root_log2order is not None else nt.modulus_order(m)

    def staging(self, n: int):
        """One pinned host block of rows f, g and the result for a request of
        length n."""
        return self.torch.empty((3, n), dtype=self.dtype, pin_memory=True)

    def operand_views(self, staged):
        v = staged.numpy().view(self.np_dtype)
        return v[0], v[1]

    def prepare(self, f: np.ndarray, g: np.ndarray):
        """Runs on the submitting thread: pinned host copies of the operands
        and a pinned buffer for the result."""
        t = self.staging(f.size)
        vf, vg = self.operand_views(t)
        vf[...] = f
        vg[...] = g
        return t

    def launch(self, reqs, stream_id: int):
        """Copies operands in, runs one conv_batched over the requests, copies
        results out; returns a handle to poll."""
        torch, nt = self.torch, self.nt
        s = self.streams[stream_id]
        k = len(reqs)
        for r in reqs:        # the copies below address whole staging blocks by raw pointer
            t = r.staged
            if tuple(t.shape) != (3, 1 << r.log2n) or t.dtype != self.dtype or not t.is_contiguous():
                raise ValueError("request %d: staging block is not a (3, %d) block of this executor"
                                 % (r.rid, 1 << r.log2n))
        off = np.fromiter((r.offset for r in reqs), np.uint64, k)
        lg = np.fromiter((r.log2n for r in reqs), np.uint64, k)
        host = np.fromiter((r.staged.data_ptr() for r in reqs), np.uint64, k)
        nb = (np.uint64(1) << lg) * np.uint64(self.wb)                  # bytes of one row
        dev_off = off * np.uint64(self.wb)
        # one library call uploads every request's f and g rows, one downloads h
        up_dst = np.concatenate([self.F_ptr + dev_off, self.G_ptr + dev_off])
        up_src = np.concatenate([host, host + nb])
        down_dst = host + nb * np.uint64(2)
        down_src = self.H_ptr + dev_off
        with torch.cuda.stream(s):
            nt.copy_batch(up_dst, up_src, np.concatenate([nb, nb]), stream=s)
            desc = nt.BatchDesc(lg.astype(np.uint8), off)
            # a served batch's descriptor is used once: the stream's staging ring
            nt.conv_batched(self.F, self.G, desc, self.m, root=self.root, root_log2order=self.rlo, out=self.H,
                            flags=nt.FLAG_TRANSIENT, stream=s)
            nt.copy_batch(down_dst, down_src, nb, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        # the staging blocks stay referenced by the handle until the event has
        # passed, and afterwards by the result arrays
        return (ev, [r.staged for r in reqs], desc)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        # views of the pinned result rows: the staging block lives as long as
        # the caller keeps the array
        return [t[2].numpy().view(self.np_dtype) for t in handle[1]]


class ConvServer:
    """Continuous-batching server over an executor (see module docstring)."""

    def __init__(self, executor, capacity_log2: int, min_log2: int = 0, max_batch: int = 512,
                 max_inflight: int = 4, max_batch_elems: int | None = None, solo_log2n: int = 16):
        """max_batch caps the requests of one launch; max_batch_elems caps its
        arena elements (a single larger request still goes alone), so that
        several batches fit in the arena at once and the uploads of one
        overlap the work of another.  Requests of 2^solo_log2n words and more
        run as batches of their own (0: never), as in the native scheduler: in
        a batch with other items a long convolution runs on one workgroup and
        the whole batch completes with it."""
        self.ex = executor
        self.alloc = BuddyAllocator(capacity_log2, min_log2)
        self.max_batch = max_batch
        self.max_batch_elems = max_batch_elems
        self.max_inflight = max_inflight
        self.solo_log2n = solo_log2n
        self.queue = collections.deque()
        self.inflight = []
        self.stats = ServeStats()
        self._next_stream = 0
        self._rid = 0
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._stop = False
        self._thread = None
        self._outstanding = 0       # submitted and not yet completed, failed or cancelled
        self.admission_log = collections.deque(maxlen=STATS_WINDOW)     # request ids in admission order (the latest)

    # ------------------------------------------------------------ client side
    def _log2_len(self, n: int) -> int:
        if n <= 0 or n & (n - 1):
            raise ValueError("request length must be a power of two")
        log2n = int(n).bit_length() - 1
        if log2n > self.alloc.total_log2:
            raise ValueError("request larger than the device arena")
        return log2n

    def submit(self, f: np.ndarray, g: np.ndarray) -> concurrent.futures.Future:
        if f.shape != g.shape or f.ndim != 1:
            raise ValueError("f and g must be 1-D of the same power-of-two length")
        log2n = self._log2_len(f.size)
        arrival = time.monotonic()
        return self._enqueue(self.ex.prepare(f, g), log2n, arrival)

    def buffers(self, n: int):
        """Zero-copy submission, first half: returns (f, g, token), where f and g
        are writable host arrays of length n inside a staging buffer.  Fill
        them, then call submit_staged(token) once."""
        log2n = self._log2_len(n)
        staged = self.ex.staging(n)
        f, g = self.ex.operand_views(staged)
        return f, g, StagedToken(staged, log2n)

    def submit_staged(self, token: StagedToken) -> concurrent.futures.Future:
        """Zero-copy submission, second half: enqueues the filled buffer."""
        if token.used:
            raise ValueError("staging token already submitted")
        token.used = True
        return self._enqueue(token.staged, token.log2n, time.monotonic())

    def _enqueue(self, staged, log2n: int, arrival: float) -> concurrent.futures.Future:
        fut = concurrent.futures.Future()
        with self._lock:
            r = Request(self._rid, staged, log2n, arrival, fut)
            self._rid += 1
            self._outstanding += 1
            self.queue.append(r)
            self._wake.notify()
        fut.request = r
        return fut

    def cancel(self, fut) -> bool:
        """Cancels a request that has not been admitted yet."""
        with self._lock:
            r = fut.request
            if r.offset < 0 and r in self.queue:
                self.queue.remove(r)
                r.cancelled = True
                self._outstanding -= 1
                fut.cancel()
                return True
        return False

    # ------------------------------------------------------------ scheduler
    def start(self):
        self._thread = threading.Thread(target=self._run, name="conv-server", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain: bool = True):
        if drain:
            self.drain()
        with self._lock:
            self._stop = True
            self._wake.notify()
        if self._thread:
            self._thread.join()

    def drain(self, timeout: float = 600.0):
        t0 = time.monotonic()
        while True:
            with self._lock:
                if self._outstanding == 0:
                    return
            if time.monotonic() - t0 > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(0.0005)

    def _admit(self):
        """Admits queued requests in arrival order while slots are free."""
        admitted = []
        elems = 0
        while self.queue and len(admitted) < self.max_batch:
            r = self.queue[0]
            size = 1 << max(r.log2n, self.alloc.min_log2)
            solo = self.solo_log2n != 0 and r.log2n >= self.solo_log2n
            if admitted and (solo or (self.max_batch_elems is not None and elems + size > self.max_batch_elems)):
                break
            off = self.alloc.alloc(r.log2n)
            if off is None:
                break
            self.queue.popleft()
            r.offset = off
            elems += size
            admitted.append(r)
            self.admission_log.append(r.rid)
            if solo:
                break
        self.stats.peak_used = max(self.stats.peak_used, self.alloc.used)
        return admitted

    def _complete(self, b: _Batch):
        outs = self.ex.results(b.handle)
        now = time.monotonic()
        for r, o in zip(b.reqs, outs):
            r.out = o
            r.done_time = now
            self.alloc.free(r.offset, r.log2n)
            self.stats.latencies.append(now - r.arrival)
            self.stats.completed += 1
            self._outstanding -= 1
            r.future.set_result(o)

    def _run(self):
        while True:
            with self._lock:
                if self._stop:
                    return
                admitted = self._admit() if len(self.inflight) < self.max_inflight else []
            if admitted:
                sid = self._next_stream % len(self.ex.streams)
                self._next_stream += 1
                try:
                    h = self.ex.launch(admitted, sid)
                except Exception as e:          # a failed launch fails its requests only
                    with self._lock:
                        for r in admitted:
                            self.alloc.free(r.offset, r.log2n)
                            self._outstanding -= 1
                            r.future.set_exception(e)
                    continue
                with self._lock:
                    self.inflight.append(_Batch(admitted, h, sid, time.monotonic()))
                    self.stats.batch_sizes.append(len(admitted))
                    self.stats.peak_inflight = max(self.stats.peak_inflight, len(self.inflight))
            done = [b for b in list(self.inflight) if self.ex.poll(b.handle)]
            if done:
                with self._lock:
                    for b in done:
                        self.inflight.remove(b)
                        self._complete(b)
            if not admitted and not done:
                # nothing to launch or complete: sleep until a submission or the
                # next poll of the batches in flight (never spin on the lock)
                with self._lock:
                    if not self._stop:
                        self._wake.wait(timeout=0.0002)


class NativeConvServer:
    """The served form run by the library's own scheduler thread (ntt_server_*
    in the C ABI): the same admission, batching and stream rotation as
    ConvServer, with no Python on the per-request path.  submit() copies f and
    g into a pinned staging block inside the library (the interpreter lock is
    released during the call) and returns a ticket; result() waits for it.
    host_arenas=True creates the server with ntt_server_create_host: the
    request's slot is in pinned host arenas that the batch kernels read and
    write directly, with no copies between host and device."""

    def __init__(self, m: int, capacity_log2: int, elem_bits: int = 64, streams: int = 4, max_batch: int = 512,
                 max_batch_elems: int = 0, max_inflight: int = 4, root: int = 2, root_log2order: int | None = None,
                 solo_log2n: int | None = None, host_arenas: bool = False):
        import ctypes
        import paper_1005_1497_amd as nt
        self._nt, self._ct = nt, ctypes
        self.np_dtype = np.uint64 if elem_bits == 64 else np.uint32
        rlo = root_log2order if root_log2order is not None else nt.modulus_order(m)
        h = ctypes.c_void_p()
        create = nt.lib.ntt_server_create_host if host_arenas else nt.lib.ntt_server_create
        nt._check(create(m, root, rlo, elem_bits, capacity_log2, streams, max_batch, max_batch_elems, max_inflight,
                         ctypes.byref(h)), "ntt_server_create")
        self._h = h
        if solo_log2n is not None:   # else the library's default (2^16 words and more run alone)
            nt._check(nt.lib.ntt_server_set_solo(h, int(solo_log2n)), "ntt_server_set_solo")

    def submit(self, f: np.ndarray, g: np.ndarray) -> int:
        f = np.ascontiguousarray(f, dtype=self.np_dtype)
        g = np.ascontiguousarray(g, dtype=self.np_dtype)
        n = f.size
        if f.shape != g.shape or f.ndim != 1 or n == 0 or n & (n - 1):
            raise ValueError("f and g must be 1-D of the same power-of-two length")
        t = self._ct.c_uint64()
        self._nt._check(self._nt.lib.ntt_server_submit(self._h, f.ctypes.data, g.ctypes.data, n.bit_length() - 1,
                                                       self._ct.byref(t)), "ntt_server_submit")
        return (t.value, n)

    def stage(self, n: int):
        """Zero-copy submission, first half: (f, g, ticket) with f and g
        writable arrays over the pinned rows of a staging block inside the
        library.  Fill them, then call submit_staged(ticket); they are not to
        be touched after result()."""
        if n <= 0 or n & (n - 1):
            raise ValueError("request length must be a power of two")
        ct = self._ct
        fp, gp, t = ct.c_void_p(), ct.c_void_p(), ct.c_uint64()
        self._nt._check(self._nt.lib.ntt_server_stage(self._h, n.bit_length() - 1, ct.byref(fp), ct.byref(gp),
                                                      ct.byref(t)), "ntt_server_stage")
        word = ct.c_uint64 if self.np_dtype == np.uint64 else ct.c_uint32
        f = np.ctypeslib.as_array((word * n).from_address(fp.value))
        g = np.ctypeslib.as_array((word * n).from_address(gp.value))
        return f, g, (t.value, n)

    def submit_staged(self, ticket) -> None:
        self._nt._check(self._nt.lib.ntt_server_submit_staged(self._h, ticket[0]), "ntt_server_submit_staged")

    def result(self, ticket, timeout: float = -1.0, out: np.ndarray | None = None) -> np.ndarray:
        """Waits for the request and returns its result, copied into `out`
        when given (a reused buffer saves the page faults of a fresh one)."""
        tid, n = ticket
        if out is None:
            out = np.empty(n, dtype=self.np_dtype)
        elif out.dtype != self.np_dtype or out.shape != (n,) or not out.flags.c_contiguous:
            raise ValueError("out must be a contiguous array of %d words" % n)
        self._nt._check(self._nt.lib.ntt_server_wait(self._h, tid, out.ctypes.data, timeout), "ntt_server_wait")
        return out

    def stats(self, reset: bool = False) -> dict:
        ct = self._ct
        c, mb, p50, p99 = ct.c_uint64(), ct.c_double(), ct.c_double(), ct.c_double()
        self._nt._check(self._nt.lib.ntt_server_stats(self._h, ct.byref(c), ct.byref(mb), ct.byref(p50),
                                                      ct.byref(p99), 1 if reset else 0), "ntt_server_stats")
        return {"completed": c.value, "mean_batch": mb.value, "p50_ms": p50.value, "p99_ms": p99.value}

    def close(self):
        if self._h:
            self._nt.lib.ntt_server_destroy(self._h)
            self._h = None

    def __del__(self):
        if getattr(self, "_h", None):
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
