"""Row batches streamed from host memory: A larger than device memory.

The product is a sum over row batches (Sec. III-B, Eqs. (3)-(4)): batch l
holds the IDs in [l m~, (l+1) m~) of every set and B is the sum of the
batches' Gram products.  Here the sets stay in host memory and are cut into
parts, each an ID range of 2^(U - part_bits) rows (one or more batches).  A
producer thread gathers part p + 1 into page-locked memory and copies it to
the GPU on its own stream while the caller's thread encodes part p and adds
its counts into the resident B (jas_gram with JAS_ACCUMULATE; the part's IDs
relabelled to offsets in its range, so it is encoded over 2^(U - part_bits)
rows); jas_finalize
then writes the diagonal, the unions and J.  Two staging slots in host and
device memory alternate, so the device holds two parts' IDs, one part's
encoding and B at any time.

Every set must list its IDs in ascending order (as k-mer files sorted by
k-mer do): a part is then one contiguous slice of each set, found by binary
search.  All arithmetic runs in the HIP library; this module only plans the
slices, copies memory and orders the streams.
"""
from __future__ import annotations

import queue
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import jas as cabi


def plan_parts(ids: np.ndarray, offsets: np.ndarray, universe_bits: int, part_bits: int,
               check_sorted: bool = True) -> np.ndarray:
    """bounds[p, i] .. bounds[p + 1, i]: the entries of set i whose ID lies in
    part p, i.e. in [p << s, (p + 1) << s) with s = universe_bits - part_bits."""
    U, pb = int(universe_bits), int(part_bits)
    if not 1 <= U <= 63 or not 0 <= pb <= min(U, 20):
        raise ValueError("need 1 <= universe_bits <= 63 and 0 <= part_bits <= min(universe_bits, 20)")
    off = np.asarray(offsets, dtype=np.uint64)
    n = off.size - 1
    cuts = np.arange((1 << pb) + 1, dtype=np.uint64) << np.uint64(U - pb)
    bounds = np.empty(((1 << pb) + 1, n), dtype=np.uint64)
    for i in range(n):
        a, b = int(off[i]), int(off[i + 1])
        seg = ids[a:b]
        if check_sorted and seg.size > 1 and np.any(seg[1:] < seg[:-1]):
            raise ValueError(f"set {i}: IDs are not in ascending order")
        if seg.size and int(seg[-1]) >> U:
            raise ValueError(f"set {i}: an ID is >= 2^universe_bits")
        bounds[:, i] = a + np.searchsorted(seg, cuts, side="left").astype(np.uint64)
    return bounds


def _gather(ids, lo, hi, dst, pool, chunks, base: int = 0):
    """dst <- concatenation of ids[lo[i]:hi[i]] - base over i; returns the CSR offsets."""
    sizes = (hi - lo).astype(np.int64)
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    b = np.uint64(base)

    def work(r):
        for i in range(r[0], r[1]):
            if sizes[i]:
                np.subtract(ids[int(lo[i]):int(hi[i])], b, out=dst[off[i]:off[i + 1]])

    n = sizes.size
    step = max(1, -(-n // chunks))
    list(pool.map(work, [(s, min(n, s + step)) for s in range(0, n, step)]))
    return off


def all_pairs_streamed(ids: np.ndarray, offsets: np.ndarray, universe_bits: int, part_bits: int,
                       batch_bits: int = 0, dense_min_degree: int = 0, upper: bool = False, gram_flags: int = 0,
                       check_sorted: bool = True, workers: int = 8, bounds: np.ndarray = None):
    """Exact B, |X_i|, C and J of all set pairs, streaming the sets from host memory.

    ids, offsets: host arrays (uint64), CSR, each set ascending.  Returns a dict
    of device tensors B (int32), card (int64), den (int64), J (float64) in the
    full (n*n) or upper layout, plus per-part encode stats and host timings."""
    import torch

    ids = np.asarray(ids)
    if ids.dtype != np.uint64:
        raise TypeError("ids must be uint64")
    n = int(np.asarray(offsets).size - 1)
    if bounds is None:
        bounds = plan_parts(ids, offsets, universe_bits, part_bits, check_sorted)
    nparts = bounds.shape[0] - 1
    # a part's IDs are relabelled to their offset in the part's range, so each
    # part is encoded over its own 2^(U - part_bits) rows: the sort's top-bit
    # buckets then split the part's IDs, not the whole universe's
    part_bits = (nparts - 1).bit_length()
    part_shift = universe_bits - part_bits
    part_U = max(1, part_shift)
    part_len = (bounds[1:] - bounds[:-1]).sum(axis=1).astype(np.int64)
    cap = max(1, int(part_len.max(initial=0)))
    dev = torch.device("cuda", torch.cuda.current_device())
    length = n * (n + 1) // 2 if upper else n * n
    B = torch.zeros(length, dtype=torch.int32, device=dev)
    card = torch.zeros(max(n, 1), dtype=torch.int64, device=dev)[:n]
    den = torch.empty(length, dtype=torch.int64, device=dev)
    J = torch.empty(length, dtype=torch.float64, device=dev)
    compute = torch.cuda.current_stream()
    copy = torch.cuda.Stream()
    slots = 2
    host = [torch.empty(cap, dtype=torch.int64, pin_memory=True) for _ in range(slots)]
    host_off = [torch.empty(n + 1, dtype=torch.int64, pin_memory=True) for _ in range(slots)]
    dids = [torch.empty(cap, dtype=torch.int64, device=dev) for _ in range(slots)]
    doff = [torch.empty(n + 1, dtype=torch.int64, device=dev) for _ in range(slots)]
    copied = [torch.cuda.Event() for _ in range(slots)]
    used = [None] * slots  # event after the part in the slot was encoded
    free = [threading.Semaphore(1) for _ in range(slots)]
    ready: queue.Queue = queue.Queue()
    stop = threading.Event()
    t_gather = [0.0]
    errors = []

    def producer():
        try:
            with ThreadPoolExecutor(max_workers=workers) as pool:
                for p in range(nparts):
                    k = p % slots
                    free[k].acquire()  # the consumer has queued its use of slot k
                    if stop.is_set():
                        return
                    with torch.cuda.stream(copy):
                        if used[k] is not None:
                            copied[k].synchronize()   # the host slot's last copy has landed
                            copy.wait_event(used[k])  # the device slot is no longer read
                        t0 = time.perf_counter()
                        o = _gather(ids, bounds[p], bounds[p + 1], host[k].numpy().view(np.uint64), pool, workers,
                                    base=p << part_shift)
                        host_off[k].numpy()[:] = o
                        t_gather[0] += time.perf_counter() - t0
                        L = int(o[-1])
                        if L:
                            dids[k][:L].copy_(host[k][:L], non_blocking=True)
                        doff[k].copy_(host_off[k], non_blocking=True)
                        copied[k].record(copy)
                    ready.put((p, k, L))
        except BaseException as e:  # handed to the consumer
            errors.append(e)
            ready.put(None)

    th = threading.Thread(target=producer, daemon=True)
    t0 = time.perf_counter()
    th.start()
    stats = []
    flags = gram_flags | cabi.JAS_ACCUMULATE | (cabi.JAS_UPPER if upper else 0)
    ok = False
    try:
        for _ in range(nparts):
            item = ready.get()
            if item is None:
                raise errors[0]
            p, k, L = item
            compute.wait_event(copied[k])
            opts = cabi.jas_encode_opts(part_U, min(batch_bits, part_U) if batch_bits else 0, dense_min_degree, 0, 0)
            db, st = cabi.jas_encode(dids[k], doff[k], n, opts, compute)
            cabi.jas_gram(db, flags, compute, B, card)
            ev = torch.cuda.Event()
            ev.record(compute)
            used[k] = ev
            free[k].release()
            db.close()
            st["part"], st["part_ids"] = p, L
            stats.append(st)
        ok = True
    finally:
        if not ok:
            stop.set()
            for f in free:
                f.release()
        th.join()
    cabi.jas_finalize(n, cabi.JAS_UPPER if upper else 0, compute, B, card, den, J)
    return {"B": B, "card": card, "den": den, "J": J, "parts": stats, "n_parts": nparts,
            "max_part_ids": cap, "host_gather_s": t_gather[0], "wall_s_to_last_launch": time.perf_counter() - t0}
