"""Thin Python binding of the C ABI in include/kkt.h (argument marshalling only).

Every step of the factorization and the solves runs in the HIP library
``libkkt.so``; PyTorch only provides device memory and the stream.  Importing
this module fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkkt.so")

KKT_OK = 0
KKT_EDIMS, KKT_EPOINTER, KKT_EWORKSPACE, KKT_ELAUNCH, KKT_ENOTFACTORED = -1, -2, -3, -4, -5
MAX_B, MAX_NG, MAX_NRHS = 48, 16, 8
NUM_CLASSES = 5
CLASS_BLOCKS = (8, 16, 24, 32, 48)
WS_FOREIGN = 2


class Dims(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("b", ctypes.c_int32), ("ng", ctypes.c_int32),
                ("p", ctypes.c_int32), ("N1", ctypes.c_int32)]


MAX_LEVELS = 4


class Nest(ctypes.Structure):
    """Recursive segmentation of one system: p[l] segments of the level-l reduced
    chain (0 ends it), N1[l] its first-segment length (0: Eq. 13's balance)."""
    _fields_ = [("p", ctypes.c_int32 * MAX_LEVELS), ("N1", ctypes.c_int32 * MAX_LEVELS)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("num_systems", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("num_items", ctypes.c_int32),
                ("num_classes", ctypes.c_int32), ("D_len", ctypes.c_int64), ("C_len", ctypes.c_int64),
                ("B_len", ctypes.c_int64), ("corner_len", ctypes.c_int64), ("rhs_len", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("solve_flops", ctypes.c_double), ("factor_words", ctypes.c_int64),
                ("input_words", ctypes.c_int64)]


class SystemLayout(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("b", ctypes.c_int32), ("ng", ctypes.c_int32), ("p", ctypes.c_int32),
                ("N1", ctypes.c_int32), ("Nk", ctypes.c_int32),
                ("off_D", ctypes.c_int64), ("off_C", ctypes.c_int64), ("off_B", ctypes.c_int64),
                ("off_corner", ctypes.c_int64), ("off_rhs", ctypes.c_int64),
                ("off_Ld", ctypes.c_int64), ("off_Lc", ctypes.c_int64), ("off_Lb", ctypes.c_int64),
                ("off_Lg", ctypes.c_int64), ("off_fill", ctypes.c_int64), ("off_H", ctypes.c_int64)]


class CostModel(ctypes.Structure):
    """Per padded block-size class (8, 16, 24, 32, 48): stage times of first segments,
    fill-carrying segments and reduced stages, item overhead, concurrent items of
    unsegmented systems (workers) and of segmented ones (workers_seg, 0 = workers),
    the fixed cost of one more level of recursive segmentation (t_level;
    64 t_first when a dict leaves it out), and the sweep family per class (family:
    0 library choice, 1 dense 32-wide tiles, 2 row-lane; 0 when left out)."""
    _fields_ = [("t_first", ctypes.c_double * NUM_CLASSES), ("t_fill", ctypes.c_double * NUM_CLASSES),
                ("t_red", ctypes.c_double * NUM_CLASSES), ("t_item", ctypes.c_double * NUM_CLASSES),
                ("workers", ctypes.c_double * NUM_CLASSES), ("workers_seg", ctypes.c_double * NUM_CLASSES),
                ("t_level", ctypes.c_double * NUM_CLASSES), ("family", ctypes.c_double * NUM_CLASSES)]

    @classmethod
    def from_dict(cls, d):
        m = cls()
        d = dict(d)
        if "t_level" not in d:
            d["t_level"] = [64.0 * float(v) for v in d.get("t_first", [0.0] * NUM_CLASSES)]
        for k in ("t_first", "t_fill", "t_red", "t_item", "workers", "workers_seg", "t_level", "family"):
            vals = list(d.get(k, [0.0] * NUM_CLASSES))
            if len(vals) != NUM_CLASSES:
                raise ValueError("cost model field %s needs %d entries, got %d" % (k, NUM_CLASSES, len(vals)))
            for i, v in enumerate(vals):
                getattr(m, k)[i] = float(v)
        return m


class QPData(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("Q", "S", "T", "Qg", "EL", "ER", "EG", "IL", "IR", "IG", "w")]


class KKTError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded ``libkkt.so`` (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libkkt.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.kkt_plan_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Dims), i32]
        L.kkt_plan_create_tuned.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Dims), i32,
                                            ctypes.POINTER(CostModel)]
        L.kkt_plan_create_nested.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Dims), ctypes.POINTER(Nest),
                                             i32, ctypes.POINTER(CostModel)]
        L.kkt_plan_reduced.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.kkt_plan_destroy.argtypes = [vp]
        L.kkt_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.kkt_plan_system.argtypes = [vp, i32, ctypes.POINTER(SystemLayout)]
        L.kkt_plan_factor_offset.argtypes = [vp]
        L.kkt_plan_factor_offset.restype = i64
        L.kkt_workspace_init.argtypes = [vp, vp, vp]
        L.kkt_factor.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.kkt_solve.argtypes = [vp, vp, vp, vp]
        L.kkt_factor_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.kkt_factor_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.kkt_solve_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.kkt_plan_class_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                          ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.kkt_plan_set_class_events.argtypes = [vp, i32, vp, vp]
        L.kkt_plan_class_kind.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.kkt_workspace_error.argtypes = [vp, vp, vp, ctypes.POINTER(i32)]
        L.kkt_ragged_create.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(vp)]
        L.kkt_ragged_destroy.argtypes = [vp]
        L.kkt_ragged_lengths.argtypes = [vp] + [ctypes.POINTER(i64)] * 5
        L.kkt_ragged_pad.argtypes = [vp] * 11 + [vp]
        L.kkt_ragged_unpad.argtypes = [vp, vp, vp, vp]
        L.kkt_qp_create.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(vp)]
        L.kkt_qp_destroy.argtypes = [vp]
        L.kkt_qp_lengths.argtypes = [vp] + [ctypes.POINTER(i64)] * 9
        L.kkt_qp_offsets.argtypes = [vp, i32, ctypes.POINTER(i64)]
        dbl = ctypes.c_double
        L.kkt_qp_assemble.argtypes = [vp, ctypes.POINTER(QPData), dbl, dbl, vp, vp, vp, vp, vp]
        L.kkt_qp_reduce_rhs.argtypes = [vp, ctypes.POINTER(QPData), dbl, vp, vp, vp, vp, vp]
        L.kkt_qp_recover.argtypes = [vp, ctypes.POINTER(QPData), dbl, vp, vp, vp, vp, vp, vp]
        L.kkt_ipm_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
        L.kkt_ipm_destroy.argtypes = [vp]
        L.kkt_ipm_solve.argtypes = [vp, vp, ctypes.POINTER(QPData), vp, vp, vp, dbl, dbl, dbl, i32, vp, vp, vp, vp,
                                    vp, vp]
        for name in ("kkt_ragged_create", "kkt_ragged_destroy", "kkt_ragged_lengths", "kkt_ragged_pad",
                     "kkt_ragged_unpad", "kkt_qp_create", "kkt_qp_destroy", "kkt_qp_lengths", "kkt_qp_offsets",
                     "kkt_qp_assemble", "kkt_qp_reduce_rhs", "kkt_qp_recover", "kkt_ipm_create", "kkt_ipm_destroy",
                     "kkt_ipm_solve"):
            getattr(L, name).restype = ctypes.c_int
        L.kkt_status_string.restype = ctypes.c_char_p
        L.kkt_status_string.argtypes = [ctypes.c_int]
        for name in ("kkt_plan_create", "kkt_plan_create_tuned", "kkt_plan_create_nested", "kkt_plan_reduced",
                     "kkt_plan_destroy", "kkt_plan_get_info", "kkt_plan_system",
                     "kkt_workspace_init", "kkt_factor", "kkt_solve", "kkt_factor_solve", "kkt_solve_adjoint",
                     "kkt_factor_solve_noalloc", "kkt_plan_class_info", "kkt_plan_class_kind", "kkt_plan_set_class_events", "kkt_workspace_error"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


EXPORTED = ("kkt_plan_create", "kkt_plan_create_tuned", "kkt_plan_destroy", "kkt_plan_get_info", "kkt_plan_system",
            "kkt_plan_factor_offset", "kkt_workspace_init", "kkt_factor", "kkt_solve",
            "kkt_factor_solve", "kkt_solve_adjoint", "kkt_status_string", "kkt_plan_class_info",
            "kkt_plan_class_kind", "kkt_plan_set_class_events", "kkt_workspace_error", "kkt_factor_solve_noalloc",
            "kkt_ragged_create", "kkt_ragged_destroy", "kkt_ragged_lengths", "kkt_ragged_pad", "kkt_ragged_unpad",
            "kkt_plan_create_nested", "kkt_plan_reduced", "kkt_qp_create", "kkt_qp_destroy", "kkt_qp_lengths",
            "kkt_qp_offsets", "kkt_qp_assemble", "kkt_qp_reduce_rhs", "kkt_qp_recover", "kkt_ipm_create",
            "kkt_ipm_destroy", "kkt_ipm_solve")

# bytes of the no-allocation entry point's device array (plans above it are refused)
NOALLOC_MAX_BYTES = 32 << 20


def _check(rc, what):
    if rc != KKT_OK:
        raise KKTError("%s failed: %s (%d)" % (what, lib().kkt_status_string(rc).decode(), rc))


def _ptr(t):
    """Device pointer of a float64 / int32 / uint8 CUDA tensor, or None for an empty one."""
    if t is None or t.numel() == 0:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A plan for a batch of systems: ``dims`` is a list of (N, b, ng[, p[, N1]]).

    p = 0 lets the plan choose the segment count (and the recursion of the reduced
    chain) from ``cost_model`` (a ``CostModel`` or a dict of its fields; None = the
    default model).  ``nest``: per system None or a sequence of segment counts of
    its reduced chain, that chain's reduced chain, ... (recursive segmentation;
    read for systems with a given p); an entry may be a pair (p, N1) to fix that
    level's first-segment length."""

    def __init__(self, dims, nrhs=1, cost_model=None, nest=None, _borrow=None):
        if _borrow is not None:
            self._h, self._owned = _borrow, False
            self._load(int(nrhs))
            return
        dims = [tuple(d) for d in dims]
        arr = (Dims * len(dims))()
        for i, d in enumerate(dims):
            N, b, ng = int(d[0]), int(d[1]), int(d[2])
            p = int(d[3]) if len(d) > 3 else 1
            N1 = int(d[4]) if len(d) > 4 else 0
            arr[i] = Dims(N, b, ng, p, N1)
        h = ctypes.c_void_p()
        if nest is not None:
            if len(nest) != len(dims):
                raise ValueError("nest needs one entry per system")
            narr = (Nest * len(dims))()
            for i, ps in enumerate(nest):
                ps = list(ps or [])
                if len(ps) > MAX_LEVELS:
                    raise ValueError("at most %d levels of recursion" % MAX_LEVELS)
                for l, q in enumerate(ps):
                    q, n1 = (q if isinstance(q, (tuple, list)) else (q, 0))
                    narr[i].p[l] = int(q)
                    narr[i].N1[l] = int(n1)
            cm = None
            if cost_model is not None:
                cm = cost_model if isinstance(cost_model, CostModel) else CostModel.from_dict(cost_model)
            _check(lib().kkt_plan_create_nested(ctypes.byref(h), len(dims), arr, narr, int(nrhs),
                                                ctypes.byref(cm) if cm is not None else None),
                   "kkt_plan_create_nested")
        elif cost_model is None:
            _check(lib().kkt_plan_create(ctypes.byref(h), len(dims), arr, int(nrhs)), "kkt_plan_create")
        else:
            cm = cost_model if isinstance(cost_model, CostModel) else CostModel.from_dict(cost_model)
            _check(lib().kkt_plan_create_tuned(ctypes.byref(h), len(dims), arr, int(nrhs), ctypes.byref(cm)),
                   "kkt_plan_create_tuned")
        self._h, self._owned = h, True
        self._load(int(nrhs))

    def _load(self, nrhs):
        h = self._h
        self.nrhs = nrhs
        info = PlanInfo()
        _check(lib().kkt_plan_get_info(h, ctypes.byref(info)), "kkt_plan_get_info")
        self.info = info
        self.S = int(info.num_systems)
        self.factor_offset = int(lib().kkt_plan_factor_offset(h))
        self.layouts = []
        for s in range(self.S):
            lay = SystemLayout()
            _check(lib().kkt_plan_system(h, s, ctypes.byref(lay)), "kkt_plan_system")
            self.layouts.append(lay)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and getattr(self, "_owned", False) and _lib is not None:
            _lib.kkt_plan_destroy(h)
            self._h = None

    def reduced(self, s):
        """(child plan, child system, workspace byte offset) where the reduced chain
        of system s is factored when it is segmented, else None.  The child plan is
        owned by this one (kept alive by the returned view's reference)."""
        ch, cs, off = ctypes.c_void_p(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().kkt_plan_reduced(self._h, int(s), ctypes.byref(ch), ctypes.byref(cs), ctypes.byref(off)),
               "kkt_plan_reduced")
        if not ch.value:
            return None
        view = Plan(None, self.nrhs, _borrow=ch)
        view._parent = self
        return view, int(cs.value), int(off.value)

    def nest_depth(self, s):
        """Levels of recursive segmentation below system s (0: its chain, if any, is swept sequentially)."""
        r = self.reduced(s)
        return 0 if r is None else 1 + r[0].nest_depth(r[1])

    # ---- memory
    def pool_lengths(self):
        i = self.info
        return dict(D=i.D_len, C=i.C_len, B=i.B_len, corner=i.corner_len, rhs=i.rhs_len)

    def new_workspace(self, device="cuda", stream=None):
        import torch
        ws = torch.empty(int(self.info.workspace_bytes) + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        ws = ws[off:off + int(self.info.workspace_bytes)]
        self.init_workspace(ws, stream)
        return ws

    def init_workspace(self, ws, stream=None):
        self._check_ws(ws)
        _check(lib().kkt_workspace_init(self._h, _ptr(ws), _stream(stream)), "kkt_workspace_init")

    def _check_ws(self, ws):
        import torch
        if ws.dtype != torch.uint8 or ws.numel() < self.info.workspace_bytes:
            raise ValueError("workspace must be a uint8 device tensor of >= %d bytes" % self.info.workspace_bytes)

    def _check_pool(self, t, name):
        import torch
        n = self.pool_lengths()[name]
        if n == 0:
            return
        if t is None or t.dtype != torch.float64 or t.numel() < n:
            raise ValueError("%s must be a float64 device tensor with >= %d elements" % (name, n))

    # ---- calls
    def factor(self, D, C, B, corner, ws, info, stream=None):
        for t, n in ((D, "D"), (C, "C"), (B, "B"), (corner, "corner")):
            self._check_pool(t, n)
        self._check_ws(ws)
        _check(lib().kkt_factor(self._h, _ptr(D), _ptr(C), _ptr(B), _ptr(corner), _ptr(ws), _ptr(info),
                                _stream(stream)), "kkt_factor")

    def factor_solve(self, D, C, B, corner, ws, rhs, info, stream=None):
        for t, n in ((D, "D"), (C, "C"), (B, "B"), (corner, "corner"), (rhs, "rhs")):
            self._check_pool(t, n)
        self._check_ws(ws)
        _check(lib().kkt_factor_solve(self._h, _ptr(D), _ptr(C), _ptr(B), _ptr(corner), _ptr(ws), _ptr(rhs),
                                      _ptr(info), _stream(stream)), "kkt_factor_solve")

    def factor_solve_noalloc(self, D, C, B, corner, rhs, info, stream=None):
        """factor_solve with the library's own device array as the workspace: no
        allocation; calls that overlap on one device race."""
        for t, n in ((D, "D"), (C, "C"), (B, "B"), (corner, "corner"), (rhs, "rhs")):
            self._check_pool(t, n)
        _check(lib().kkt_factor_solve_noalloc(self._h, _ptr(D), _ptr(C), _ptr(B), _ptr(corner), _ptr(rhs),
                                              _ptr(info), _stream(stream)), "kkt_factor_solve_noalloc")

    def solve(self, ws, rhs, stream=None):
        self._check_pool(rhs, "rhs")
        self._check_ws(ws)
        _check(lib().kkt_solve(self._h, _ptr(ws), _ptr(rhs), _stream(stream)), "kkt_solve")

    def solve_adjoint(self, ws, x, gx, dD, dC, dB, dcorner, stream=None):
        for t, n in ((x, "rhs"), (gx, "rhs"), (dD, "D"), (dC, "C"), (dB, "B"), (dcorner, "corner")):
            self._check_pool(t, n)
        self._check_ws(ws)
        _check(lib().kkt_solve_adjoint(self._h, _ptr(ws), _ptr(x), _ptr(gx), _ptr(dD), _ptr(dC), _ptr(dB),
                                       _ptr(dcorner), _stream(stream)), "kkt_solve_adjoint")

    # ---- reading the factor back (host side, for inspection and tests)
    def factor_blocks(self, ws_host, s):
        """Dict {(row, col): block} of hat L for system s, from a host copy (numpy
        uint8 array) of the workspace.  Labels are natural 0-based stage indices,
        'g' for the global block."""
        lay = self.layouts[s]
        F = np.frombuffer(ws_host[self.factor_offset:].tobytes(), dtype=np.float64)
        N, b, ng, p, N1, Nk = lay.N, lay.b, lay.ng, lay.p, lay.N1, lay.Nk
        b2 = b * b
        seps = [N1 + (k - 2) * (Nk + 1) for k in range(2, p + 1)]
        sepset = set(seps)
        out = {}
        for st in range(N):
            out[(st, st)] = F[lay.off_Ld + st * b2: lay.off_Ld + (st + 1) * b2].reshape(b, b)
            if ng:
                out[("g", st)] = F[lay.off_Lb + st * ng * b: lay.off_Lb + (st + 1) * ng * b].reshape(ng, b)
        for st in range(N - 1):
            blk = F[lay.off_Lc + st * b2: lay.off_Lc + (st + 1) * b2].reshape(b, b)
            out[(st, st + 1) if st in sepset else (st + 1, st)] = blk
        red = self.reduced(s)
        for k in range(2, p + 1):
            sep = seps[k - 2]
            first = sep + 1
            for i in range(2, Nk + 1):
                o = lay.off_fill + ((k - 2) * (Nk - 1) + (i - 2)) * b2
                out[(sep, first + i - 1)] = F[o:o + b2].reshape(b, b)
            if k < p and red is None:
                o = lay.off_H + (k - 2) * b2
                out[(seps[k - 1], sep)] = F[o:o + b2].reshape(b, b)
        if ng and red is None:
            out[("g", "g")] = F[lay.off_Lg: lay.off_Lg + ng * ng].reshape(ng, ng)
        if red is not None:
            # the reduced chain's factor (its stage j is separator seps[j]) replaces
            # the blocks of the separators and the corner
            child, cs, off = red
            cb = child.factor_blocks(ws_host[off:off + int(child.info.workspace_bytes)], cs)
            lab = lambda v: v if v == "g" else seps[v]
            for st in seps:
                out.pop((st, st), None)
                out.pop(("g", st), None)
            for (ri, cj), blk in cb.items():
                out[(lab(ri), lab(cj))] = blk
        return out

    def classes(self, with_grid=False):
        """[(padded block size, items, threads, lds bytes[, workgroups])] per launch class (its first launch)."""
        out = []
        for c in range(self.info.num_classes):
            bp, it, nt, lds, gr = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(),
                                   ctypes.c_int32())
            _check(lib().kkt_plan_class_info(self._h, c, ctypes.byref(bp), ctypes.byref(it), ctypes.byref(nt),
                                             ctypes.byref(lds), ctypes.byref(gr)), "kkt_plan_class_info")
            t = (bp.value, it.value, nt.value, lds.value)
            out.append(t + (gr.value,) if with_grid else t)
        return out

    def class_kinds(self):
        """Kind of each launch class: 0 row-lane, 1 dense (whole systems), 2 dense segmented."""
        out = []
        for c in range(self.info.num_classes):
            k = ctypes.c_int32()
            _check(lib().kkt_plan_class_kind(self._h, c, ctypes.byref(k)), "kkt_plan_class_kind")
            out.append(k.value)
        return out

    def workspace_error(self, ws, stream=None):
        """WS_FOREIGN if the last call on ws found another plan's tables there (its kernels
        then returned without touching their outputs), else 0."""
        f = ctypes.c_int32()
        _check(lib().kkt_workspace_error(self._h, _ptr(ws), _stream(stream), ctypes.byref(f)), "kkt_workspace_error")
        return int(f.value)

    def set_class_events(self, c, start, stop):
        """start / stop: raw hipEvent_t handles (ints) or None."""
        _check(lib().kkt_plan_set_class_events(self._h, c, ctypes.c_void_p(start), ctypes.c_void_p(stop)),
               "kkt_plan_set_class_events")

    def segments(self):
        """Segment count p chosen for every system."""
        return [lay.p for lay in self.layouts]

    def segment_lengths(self, s):
        lay = self.layouts[s]
        return [lay.N1] + [lay.Nk] * (lay.p - 1)


class Ragged:
    """Non-uniform stage sizes on top of a plan whose systems have b >= every n_i:
    ``sizes`` lists, per system of the plan, its N stage sizes.  pad() writes the
    plan's padded pools from the non-uniform ones, unpad() the real entries of a
    padded solution back (both on the device, in the library's kernels)."""

    def __init__(self, plan, sizes):
        flat = [int(n) for per in sizes for n in per]
        arr = (ctypes.c_int32 * max(1, len(flat)))(*flat)
        h = ctypes.c_void_p()
        _check(lib().kkt_ragged_create(plan._h, arr, ctypes.byref(h)), "kkt_ragged_create")
        self._h = h
        self.plan = plan
        lens = [ctypes.c_int64() for _ in range(5)]
        _check(lib().kkt_ragged_lengths(h, *[ctypes.byref(x) for x in lens]), "kkt_ragged_lengths")
        self.lengths = dict(zip(("D", "C", "B", "corner", "rhs"), (int(x.value) for x in lens)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.kkt_ragged_destroy(h)
            self._h = None

    def pad(self, src, dst, stream=None):
        """src: non-uniform pools {D, C, B, corner, r}; dst: the plan's pools (device)."""
        _check(lib().kkt_ragged_pad(self._h, _ptr(src["D"]), _ptr(src["C"]), _ptr(src["B"]), _ptr(src["corner"]),
                                    _ptr(src["r"]), _ptr(dst["D"]), _ptr(dst["C"]), _ptr(dst["B"]),
                                    _ptr(dst["corner"]), _ptr(dst["r"]), _stream(stream)), "kkt_ragged_pad")

    def unpad(self, xp, x, stream=None):
        _check(lib().kkt_ragged_unpad(self._h, _ptr(xp), _ptr(x), _stream(stream)), "kkt_ragged_unpad")


class QP:
    """KKT systems of multistage QPs (Sec. 2, Eq. 1) on a plan: assembly of Psi into
    the plan's pools, the reduced rhs and the recovery of dy, dz (kkt_qp_*).
    ``n_eq`` / ``n_in``: equality / inequality rows per constraint group, per system.
    Pools are device float64 tensors in a dict with keys Q, S, T, Qg (the plan's D,
    C, B, corner layouts), EL, ER, EG, IL, IR, IG, w."""

    NAMES = ("EL", "ER", "EG", "IL", "IR", "IG", "w", "ry", "rz")
    MAX_ROWS = 32

    def __init__(self, plan, n_eq, n_in):
        self.plan = plan
        ne = (ctypes.c_int32 * plan.S)(*[int(v) for v in n_eq])
        ni = (ctypes.c_int32 * plan.S)(*[int(v) for v in n_in])
        h = ctypes.c_void_p()
        _check(lib().kkt_qp_create(plan._h, ne, ni, ctypes.byref(h)), "kkt_qp_create")
        self._h = h
        vals = [ctypes.c_int64() for _ in range(9)]
        _check(lib().kkt_qp_lengths(h, *[ctypes.byref(v) for v in vals]), "kkt_qp_lengths")
        self.lengths = {k: int(v.value) for k, v in zip(self.NAMES, vals)}
        self.offsets = []
        for s in range(plan.S):
            arr = (ctypes.c_int64 * 9)()
            _check(lib().kkt_qp_offsets(h, s, arr), "kkt_qp_offsets")
            self.offsets.append({k: int(arr[j]) for j, k in enumerate(self.NAMES)})

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.kkt_qp_destroy(h)
            self._h = None

    @staticmethod
    def _data(pools):
        d = QPData()
        for k, _ in QPData._fields_:
            p = _ptr(pools.get(k))
            setattr(d, k, None if p is None else p.value)
        return d

    def assemble(self, pools, rho, delta, D, C, B, corner, stream=None):
        d = self._data(pools)
        _check(lib().kkt_qp_assemble(self._h, ctypes.byref(d), float(rho), float(delta), _ptr(D), _ptr(C), _ptr(B),
                                     _ptr(corner), _stream(stream)), "kkt_qp_assemble")

    def reduce_rhs(self, pools, delta, rx, ry, rz, rhs, stream=None):
        d = self._data(pools)
        _check(lib().kkt_qp_reduce_rhs(self._h, ctypes.byref(d), float(delta), _ptr(rx), _ptr(ry), _ptr(rz),
                                       _ptr(rhs), _stream(stream)), "kkt_qp_reduce_rhs")

    def recover(self, pools, delta, dx, ry, rz, dy, dz, stream=None):
        d = self._data(pools)
        _check(lib().kkt_qp_recover(self._h, ctypes.byref(d), float(delta), _ptr(dx), _ptr(ry), _ptr(rz), _ptr(dy),
                                    _ptr(dz), _stream(stream)), "kkt_qp_recover")


class IPM:
    """The interior-point loop of kkt_ipm_* on a plan (nrhs = 1) and its QP object:
    solve() runs it and returns the iterates (device tensors) and, per system, the
    iterations to convergence (-1 factorization failure, -2 not converged)."""

    def __init__(self, plan, qp):
        self.plan, self.qp = plan, qp
        h = ctypes.c_void_p()
        _check(lib().kkt_ipm_create(plan._h, qp._h, ctypes.byref(h)), "kkt_ipm_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.kkt_ipm_destroy(h)
            self._h = None

    def solve(self, ws, pools, c, beq, h, rho=1e-6, delta=1e-6, tol=1e-9, max_iter=60, stream=None):
        import torch
        dev = c.device
        x = torch.empty(self.plan.info.rhs_len, dtype=torch.float64, device=dev)
        y = torch.empty(self.qp.lengths["ry"], dtype=torch.float64, device=dev)
        z = torch.empty(self.qp.lengths["rz"], dtype=torch.float64, device=dev)
        s = torch.empty_like(z)
        status = torch.empty(self.plan.S, dtype=torch.int32, device=dev)
        d = QP._data(pools)
        _check(lib().kkt_ipm_solve(self._h, _ptr(ws), ctypes.byref(d), _ptr(c), _ptr(beq), _ptr(h), float(rho),
                                   float(delta), float(tol), int(max_iter), _ptr(x), _ptr(y), _ptr(z), _ptr(s),
                                   _ptr(status), _stream(stream)), "kkt_ipm_solve")
        return dict(x=x, y=y, z=z, s=s, status=status)


def pack_to_device(pools, device="cuda"):
    """Move numpy pools (from ``workloads.pack``) to device float64 tensors."""
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device=device, dtype=torch.float64)
            for k, v in pools.items()}
