"""Many column IDs of uneven sizes: one persistent launch (id_factor_batched), or
all items advanced in lock step (id_factor_lockstep).

A :class:`BatchedID` plan binds a list of device matrices, owns every
workspace and output buffer, and launches the batched factorization plus the
batched solve T = R11^{-1} R12 on the current stream without synchronizing, so
``run()`` can be captured in a CUDA/HIP graph (:meth:`BatchedID.capture`) and
replayed after new data has been copied into the bound inputs.
:func:`autotune` picks the workgroup size and panel width for a batch by timing
them, and caches the choice in a JSON file.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass

import torch

from . import _lib
from .api import DTYPE, _stream, colmajor, kcap_of, make_opts, round_

C = _lib.C
_ALIGN = 256


def _round_up(x: int, a: int) -> int:
    return (x + a - 1) // a * a


def _colmajor_view(buf: torch.Tensor, off: int, rows: int, cols: int, ld: int) -> torch.Tensor:
    """rows x cols column-major view (leading dimension ld) of buf[off:]."""
    return buf[off:off + ld * cols].view(cols, ld).t()[:rows]


def _bind_items(inputs, ldas, shapes, ws, kcs, dev):
    """Workspaces and output buffers of a batch, and its host descriptors."""
    w_off, r_off, p_off = [], [], []
    tw = tr = tp = 0
    for (m, n), w, kc in zip(shapes, ws, kcs):
        w_off.append(tw)
        tw += _round_up(w, _ALIGN)
        r_off.append(tr)
        tr += _round_up(max(kc, 1) * max(n, 1), 32)
        p_off.append(tp)
        tp += _round_up(max(n, 1), 64)
    bufs = {"work": torch.empty(tw + _ALIGN, dtype=torch.uint8, device=dev),
            "R": torch.zeros(tr, dtype=torch.float64, device=dev),
            "T": torch.zeros(tr, dtype=torch.float64, device=dev),
            "perm": torch.zeros(tp, dtype=torch.int32, device=dev)}
    wbase = _round_up(bufs["work"].data_ptr(), _ALIGN) - bufs["work"].data_ptr()
    items = (_lib.IdBatchItem * len(shapes))()
    for i, ((m, n), kc) in enumerate(zip(shapes, kcs)):
        it = items[i]
        it.A = inputs[i].data_ptr()
        it.m, it.n, it.lda = m, n, ldas[i]
        it.work = bufs["work"].data_ptr() + wbase + w_off[i]
        it.perm = bufs["perm"].data_ptr() + 4 * p_off[i]
        it.R = bufs["R"].data_ptr() + 8 * r_off[i]
        it.ldr = max(kc, 1)
        it.T = bufs["T"].data_ptr() + 8 * r_off[i]
        it.ldt = max(kc, 1)
    return items, bufs, r_off, p_off


def _item_results(items, shapes, kcaps, bufs, r_off, p_off):
    out = []
    for i, (m, n) in enumerate(shapes):
        k, info = int(items[i].k), int(items[i].info)
        ld = max(kcaps[i], 1)
        perm = bufs["perm"][p_off[i]:p_off[i] + n]
        R = _colmajor_view(bufs["R"], r_off[i], k, n, ld)
        solved = info in (0, C["ID_INFO_RANK_FULL"])
        T = _colmajor_view(bufs["T"], r_off[i], k if solved else 0, n - k if solved else 0, ld)
        out.append(BatchItemResult(perm, k, R, T, info))
    return out


def _bind_inputs(As):
    """(dtype, device, column-major inputs, their leading dimensions)."""
    if len(As) == 0:
        raise ValueError("empty batch")
    dtypes = {A.dtype for A in As}
    devices = {A.device for A in As}
    if len(dtypes) != 1 or len(devices) != 1:
        raise ValueError("all matrices must share dtype and device")
    dtype = dtypes.pop()
    if dtype not in DTYPE:
        raise TypeError("matrices must be float32 or float64")
    inputs, ldas = [], []
    for A in As:
        Ac, lda = colmajor(A)
        inputs.append(Ac)
        ldas.append(lda)
    return dtype, devices.pop(), inputs, ldas


@dataclass
class BatchItemResult:
    perm: torch.Tensor  # (n,) int32
    k: int
    R: torch.Tensor     # (k, n) float64, column-major view
    T: torch.Tensor     # (k, n - k) float64, column-major view (0 x 0 when not solved)
    info: int


class BatchedID:
    """Plan for the column IDs of the matrices ``As`` (same dtype and device).

    ``k`` (fixed rank) or ``tol`` (adaptive rank, ``rule``) applies to every
    item.  Matrices that are not column-major are copied once at bind time;
    :attr:`inputs` holds the tensors the kernels read (copy new data into them
    before replaying a captured graph).  ``groups``: workgroups per item --
    "auto" (shares large items so the work per workgroup evens out), an int for
    every item, or a per-item list.  ``order``: "lpt" (largest first), None
    (index order) or a permutation.
    """

    def __init__(self, As, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0,
                 block_threads=0, num_groups=0, order="lpt", groups="auto"):
        if k is not None and int(k) <= 0:
            raise ValueError("fixed rank must be >= 1")
        self.dtype, self.device, self.inputs, ldas = _bind_inputs(As)
        self.opts = make_opts(k, tol, prec, rule, k_max, nb)
        self.block_threads = int(block_threads)
        self.num_groups = int(num_groups)
        lib = _lib.load()
        shapes = [tuple(A.shape) for A in self.inputs]
        self.shapes = shapes
        self.batch = len(shapes)
        self.max_n = max(n for _, n in shapes)
        ws, kcs = [], []
        for m, n in shapes:
            w = int(lib.id_batch_item_workspace_size(m, n, ctypes.byref(self.opts)))
            if w == 0:
                raise ValueError(f"unsupported item shape {m} x {n} (the batched path takes n <= 2048)")
            ws.append(w)
            kcs.append(kcap_of(m, n, self.opts))
        self.kcaps = kcs
        items, self._bufs, self._r_off, self._p_off = _bind_items(self.inputs, ldas, shapes, ws,
                                                                  kcs, self.device)
        self.work, self.R_buf = self._bufs["work"], self._bufs["R"]
        self.T_buf, self.perm_buf = self._bufs["T"], self._bufs["perm"]
        self._items_host = items
        self._order = order
        self.cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        self.queue = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._plan_slots(groups, [None] * self.batch)

    @staticmethod
    def _cost(m, n, k):
        """Trailing-block elements read by k pivot steps (~ the work of an item)."""
        return max(m * n * k - (m + n) * k * k / 2.0 + k ** 3 / 3.0, float(m * n))

    def _plan_slots(self, groups, ks):
        """Workgroups per item and the slot list (largest first).  Costs use the
        rank ks[i] when known (e.g. from an earlier run), else kcap."""
        shapes = self.shapes
        cost = [self._cost(m, n, kc if k is None else k)
                for (m, n), kc, k in zip(shapes, self.kcaps, ks)]
        ngroups = self.cus if self.num_groups <= 0 else min(self.num_groups, self.cus)
        cap = C["ID_BATCH_MAX_GROUPS"]
        if groups == "auto":
            # large items are shared so that no workgroup carries far more than
            # an even share of the whole batch
            share = sum(cost) / max(ngroups, 1)
            self.groups = [max(1, min(cap, -(-n // 64), ngroups, int(c / share + 0.5)))
                           for c, (_, n) in zip(cost, shapes)]
        elif isinstance(groups, int):
            self.groups = [max(1, min(groups, cap, ngroups))] * self.batch
        else:
            self.groups = [max(1, min(int(g), cap, ngroups)) for g in groups]
        self._groups_mode = groups
        items = self._items_host
        for i in range(self.batch):
            items[i].groups = self.groups[i]
        raw = bytes(bytearray(items))
        self.items = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        order = self._order
        if order == "lpt":
            # largest per-workgroup share first; shared items then find their
            # workgroups free at the start
            idx = sorted(range(self.batch), key=lambda i: (-cost[i] / self.groups[i], i))
        elif order is None:
            idx = list(range(self.batch))
        else:
            idx = [int(i) for i in order]
            if sorted(idx) != list(range(self.batch)):
                raise ValueError("order must be a permutation of the item indices")
        slots = [i for i in idx for _ in range(self.groups[i])]
        self.nslots = len(slots)
        self.slots = torch.tensor(slots, dtype=torch.int32, device=self.device)

    def rebalance(self, results=None):
        """Re-plan the workgroups per item from the ranks of a finished run
        (adaptive ranks are unknown before the first one).  Call before capturing
        a graph: the plan's device arrays are replaced."""
        results = self.results() if results is None else results
        self._plan_slots(self._groups_mode, [r.k for r in results])

    def configure(self, block_threads=None, num_groups=None, nb=None):
        """Change the launch shape or panel width (workspaces do not depend on them)."""
        if block_threads is not None:
            self.block_threads = int(block_threads)
        if num_groups is not None:
            self.num_groups = int(num_groups)
        if nb is not None:
            self.opts.nb = int(nb)

    def run(self):
        """Enqueue the batched factorization and solve on the current stream."""
        if 0 < self.num_groups < max(self.groups):
            raise ValueError("num_groups is below the workgroups an item is shared by")
        lib = _lib.load()
        with torch.cuda.device(self.device):
            rc = lib.id_factor_batched(
                self.items.data_ptr(), self.batch, self.slots.data_ptr(), self.nslots,
                self.queue.data_ptr(), self.max_n, DTYPE[self.dtype], ctypes.byref(self.opts),
                self.block_threads, self.num_groups, _stream(self.device))
        _lib.check(rc, "id_factor_batched")

    def capture(self) -> torch.cuda.CUDAGraph:
        """A graph holding one run(); replay it with g.replay()."""
        side = torch.cuda.Stream(device=self.device)
        side.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(side):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        return g

    def results(self):
        """Per-item results (waits for the device)."""
        torch.cuda.synchronize(self.device)
        raw = self.items.cpu().numpy().tobytes()
        items = (_lib.IdBatchItem * self.batch).from_buffer_copy(raw)
        return _item_results(items, self.shapes, self.kcaps, self._bufs, self._r_off,
                             self._p_off)


class LockstepID:
    """Plan for the column IDs of the matrices ``As`` advanced in lock step
    (id_factor_lockstep): every launch runs one pivot step, or one panel end,
    of all unfinished items, so each launch streams the whole batch's trailing
    blocks.  Each item is the single-matrix algorithm with the same options
    (``k`` or ``tol`` and ``rule``, ``prec``, ``nb``) on its own workspace.
    ``run()`` synchronizes the stream (use :class:`BatchedID` for a launch
    that can be captured in a graph).  ``round_to`` ("f32" / "f16") selects the
    simulated single / half precision of id_factor."""

    def __init__(self, As, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0,
                 round_to=None):
        if k is not None and int(k) <= 0:
            raise ValueError("fixed rank must be >= 1")
        self.dtype, self.device, self.inputs, ldas = _bind_inputs(As)
        self.opts = make_opts(k, tol, prec, rule, k_max, nb, round_to=round_to)
        lib = _lib.load()
        self.shapes = [tuple(A.shape) for A in self.inputs]
        self.batch = len(self.shapes)
        dt = DTYPE[self.dtype]
        ws = []
        for m, n in self.shapes:
            w = int(lib.id_workspace_size(m, n, dt, ctypes.byref(self.opts)))
            if w == 0:
                raise ValueError(f"invalid item shape {m} x {n} or options")
            ws.append(w)
        self.kcaps = [kcap_of(m, n, self.opts) for m, n in self.shapes]
        self._items, self._bufs, self._r_off, self._p_off = _bind_items(
            self.inputs, ldas, self.shapes, ws, self.kcaps, self.device)
        sb = int(lib.id_lockstep_workspace_size(self._items, self.batch, dt,
                                                ctypes.byref(self.opts)))
        if sb == 0:
            raise ValueError("unsupported batch for the lock-step path (an item with more "
                             "than 49152 rows, or invalid options)")
        self.shared = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.round_to = round_to

    def run(self):
        """Factor every item and solve for T (returns when done)."""
        lib = _lib.load()
        with torch.cuda.device(self.device):
            rc = lib.id_factor_lockstep(self._items, self.batch, DTYPE[self.dtype],
                                        ctypes.byref(self.opts), self.shared.data_ptr(),
                                        self.shared.numel(), _stream(self.device))
        _lib.check(rc, "id_factor_lockstep")
        if self.round_to is not None:
            # the simulated low-precision ID keeps T rounded too (as column_id)
            for r in self.results():
                if r.T.numel():
                    round_(r.T, self.round_to)

    def results(self):
        """Per-item results of the last run()."""
        return _item_results(self._items, self.shapes, self.kcaps, self._bufs, self._r_off,
                             self._p_off)


def factor_lockstep(As, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0,
                    round_to=None):
    """Column IDs of every matrix in As advanced in lock step; list of BatchItemResult."""
    plan = LockstepID(As, k=k, tol=tol, prec=prec, rule=rule, k_max=k_max, nb=nb,
                      round_to=round_to)
    plan.run()
    return plan.results()


def factor_batched(As, k=None, tol=None, prec="f64", rule="pivot_rel", k_max=0, nb=0,
                   block_threads=0, num_groups=0):
    """Column IDs of every matrix in As in one batched call; list of BatchItemResult."""
    plan = BatchedID(As, k=k, tol=tol, prec=prec, rule=rule, k_max=k_max, nb=nb,
                     block_threads=block_threads, num_groups=num_groups)
    plan.run()
    return plan.results()


def _cache_path():
    return os.environ.get("MPID_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mpid", "batched_tune.json"))


def _signature(plan: BatchedID) -> str:
    o = plan.opts
    name = torch.cuda.get_device_name(plan.device)
    shapes = ",".join(f"{m}x{n}" for m, n in sorted(plan.shapes))
    return (f"{name}|{plan.dtype}|prec{o.prec}|rule{o.rank_rule}|k{o.k_fixed}|tol{o.rel_tol}|"
            f"kmax{o.k_max}|{shapes}")


def autotune(plan: BatchedID, candidates=None, reps: int = 3, use_cache: bool = True):
    """Time the plan under each (block_threads, nb) candidate, configure it with
    the fastest, and return {"block_threads", "nb", "ms", "table"}.  With
    groups="auto" the plan is first re-balanced from one run's ranks.  Results
    are cached by device, dtype, options and the multiset of shapes."""
    if plan._groups_mode == "auto":
        # adaptive ranks are known after one run: share the items by real work
        plan.run()
        plan.rebalance()
    key = _signature(plan)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        best = cache[key]
        plan.configure(block_threads=best["block_threads"], nb=best["nb"])
        return best
    if candidates is None:
        candidates = [(bt, nb) for bt in (256, 512) for nb in (16, 32)]
    table = []
    for bt, nb in candidates:
        plan.configure(block_threads=bt, nb=nb)
        plan.run()  # warm-up
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.run()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        times.sort()
        table.append({"block_threads": bt, "nb": nb, "ms": times[len(times) // 2]})
    best = dict(min(table, key=lambda r: r["ms"]))
    best["table"] = table
    plan.configure(block_threads=best["block_threads"], nb=best["nb"])
    if use_cache:
        cache[key] = best
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best
