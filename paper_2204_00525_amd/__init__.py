"""MI355X (gfx950) library: R of the QR decomposition of an acyclic natural
join, computed without materialising the join.

Thin ctypes binding over the C ABI in include/figaro.h.  It only marshals
arguments (device pointers of torch tensors, leading dimensions, the current
HIP stream); every step of the computation runs in the library's HIP kernels.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfigaro.so")

FIGARO_OK = 0
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOTTREE", 3: "EUNSHARED_KEY", 4: "EEMPTY_JOIN",
                5: "EOVERFLOW", 6: "ESINGULAR", 7: "ENOMEM", 8: "EHIP", 9: "EUNSUPPORTED"}
COUNT_KINDS = {"rows_per_key": 0, "theta_down": 1, "phi_circ": 2, "phi_up": 3, "phi_down": 4}


class FigaroError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"figaro status {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))


class RelationDesc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("num_keys", ctypes.c_int32),
                ("key_attr", ctypes.POINTER(ctypes.c_int32)), ("key_cols", ctypes.c_void_p),
                ("key_dtype", ctypes.c_int32), ("num_cols", ctypes.c_int32), ("parent", ctypes.c_int32)]


class PlanOptions(ctypes.Structure):
    _fields_ = [("tile_items", ctypes.c_int32), ("waves_per_task", ctypes.c_int32),
                ("keys_on_host", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("analyze_only", ctypes.c_int32), ("separate_join", ctypes.c_int32),
                ("host_plan", ctypes.c_int32)]


_lib = None


def lib():
    """Load libfigaro.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "figaro_plan_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(RelationDesc),
                                     ctypes.POINTER(PlanOptions), vp]),
        "figaro_plan_destroy": (None, [vp]),
        "figaro_plan_num_relations": (i32, [vp]),
        "figaro_plan_num_cols": (i32, [vp]),
        "figaro_plan_input_rows": (i64, [vp, i32]),
        "figaro_plan_rows": (i64, [vp, i32]),
        "figaro_plan_dropped_rows": (i64, [vp, i32]),
        "figaro_plan_join_rows": (dbl, [vp]),
        "figaro_plan_workspace_bytes": (i64, [vp]),
        "figaro_plan_permutation": (i32, [vp, i32, pi64]),
        "figaro_plan_num_groups": (i64, [vp, i32, i32]),
        "figaro_plan_group_first_rows": (i32, [vp, i32, i32, pi64]),
        "figaro_plan_counts": (i32, [vp, i32, i32, pi64]),
        "figaro_permute_values": (i32, [vp, i32, vp, i64, vp, i64, vp]),
        "figaro_unpermute_values": (i32, [vp, i32, vp, i64, vp, i64, vp]),
        "figaro_r": (i32, [vp, pp, pi64, vp, vp]),
        "figaro_r0_rows": (i64, [vp]),
        "figaro_r0": (i32, [vp, pp, pi64, vp, i64, vp, vp]),
        "figaro_last_error": (ctypes.c_char_p, [vp]),
        "figaro_profile_enable": (i32, [vp, i32]),
        "figaro_profile_read": (i32, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                      ctypes.POINTER(dbl), ctypes.POINTER(dbl)]),
        "figaro_profile_reset": (i32, [vp]),
        "figaro_debug_stack_rows": (i64, [vp]),
        "figaro_debug_stack": (i32, [vp, pp, pi64, vp, vp]),
        "figaro_debug_stack_layout": (i32, [vp, pi64, i32]),
        "figaro_debug_tile_rows": (i64, [i32, i32]),
        "figaro_debug_dense_rows": (i64, [i32, i32, i64]),
        "figaro_batch_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), i32]),
        "figaro_batch_destroy": (None, [vp]),
        "figaro_batch_stream_of": (i32, [vp, i32]),
        "figaro_r_batched": (i32, [vp, ctypes.POINTER(pp), ctypes.POINTER(pi64), pp, vp]),
        "figaro_r_backward_batched": (i32, [vp, ctypes.POINTER(pp), ctypes.POINTER(pi64), pp, pp,
                                            ctypes.POINTER(pp), ctypes.POINTER(pi64), vp]),
        "figaro_batch_capture": (i32, [vp, ctypes.POINTER(pp), ctypes.POINTER(pi64), pp, vp]),
        "figaro_batch_launch": (i32, [vp, vp]),
        "figaro_plan_create_tuned": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(RelationDesc), pp, pi64, i32,
                                           ctypes.POINTER(PlanOptions), i32, vp]),
        "figaro_plan_tuning": (i32, [vp, ctypes.POINTER(PlanOptions), ctypes.POINTER(dbl)]),
        "figaro_debug_dense_step": (i32, [i32, i64, vp, i64, i32, i64, i32, vp, i64, vp, vp]),
        "figaro_tsqr_workspace_bytes": (i64, [i64, i32]),
        "figaro_tsqr": (i32, [i64, i32, vp, i64, vp, vp, i64, vp]),
        "figaro_tsqr_noalloc": (i32, [i64, i32, vp, i64, vp, vp]),
        "figaro_svd_r": (i32, [i32, vp, vp, vp, vp, vp, vp]),
        "figaro_r_inverse": (i32, [i32, vp, vp, vp]),
        "figaro_join_multiply_workspace_bytes": (i64, [vp, i32]),
        "figaro_join_multiply": (i32, [vp, pp, pi64, vp, i64, i32, vp, i64, i64, vp, i64, vp, i64, vp, i64, vp]),
        "figaro_join_tree_cost": (i32, [i32, ctypes.POINTER(RelationDesc), i32, ctypes.POINTER(dbl), vp]),
        "figaro_choose_join_tree": (i32, [i32, ctypes.POINTER(RelationDesc), i32, ctypes.POINTER(i32),
                                          ctypes.POINTER(dbl), vp]),
    }
    optional = {
        "figaro_r_backward": (i32, [vp, pp, pi64, vp, vp, pp, pi64, vp]),
        "figaro_backward_status": (i32, [vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    for name, (res, args) in optional.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
    _lib = L
    return L


def _check(status: int, plan_handle=None):
    if status != FIGARO_OK:
        msg = lib().figaro_last_error(plan_handle)
        raise FigaroError(status, msg.decode() if msg else "")


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> int:
    return t.data_ptr()


def _device_descs(relations):
    """Relation descriptors for device key tensors; returns (descs, keepalive)."""
    import torch
    r = len(relations)
    descs = (RelationDesc * r)()
    keep = []
    for i, rel in enumerate(relations):
        attrs = np.ascontiguousarray(np.asarray(rel.key_attrs, dtype=np.int32))
        keys = rel.keys
        if keys.numel() and not keys.is_cuda:
            raise ValueError("key columns must be device tensors")
        keys = keys.contiguous()
        keep += [attrs, keys]
        descs[i].rows = int(keys.shape[1]) if keys.dim() == 2 else 0
        descs[i].num_keys = len(rel.key_attrs)
        descs[i].key_attr = attrs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        descs[i].key_cols = ctypes.c_void_p(keys.data_ptr() if keys.numel() else 0)
        descs[i].key_dtype = 8 if keys.dtype == torch.int64 else 4
        descs[i].num_cols = int(rel.ncols)
        descs[i].parent = int(rel.parent)
        if hasattr(rel, "rows_override"):
            descs[i].rows = int(rel.rows_override)
    return descs, keep


class Plan:
    """A plan over one key structure: validated join tree, reduced and sorted
    relations, exact count queries, scale factors and a device workspace.

    relations: sequence of objects with attributes key_attrs (list[int]),
    keys (torch tensor on the GPU, int32 or int64, shape (k, m)), ncols (int)
    and parent (int, -1 for the root)."""

    def __init__(self, relations: Sequence, *, tile_items: int = 0, waves_per_task: int = 0,
                 stream=None, analyze_only: bool = False, variant: int = 0, separate_join: bool = False,
                 host_plan: bool = False, _handle=None):
        L = lib()
        if analyze_only:
            self._init_host(relations, tile_items, waves_per_task)
            return
        if _handle is not None:
            self._handle = _handle
        else:
            self._handle = ctypes.c_void_p()
            descs, keep = _device_descs(relations)
            opts = PlanOptions(tile_items, waves_per_task, 0, variant, 0, int(bool(separate_join)),
                               int(bool(host_plan)))
            st = L.figaro_plan_create(ctypes.byref(self._handle), len(relations), descs, ctypes.byref(opts),
                                      _stream_handle(stream))
            del keep
            if st != FIGARO_OK:
                msg = L.figaro_last_error(None)
                raise FigaroError(st, msg.decode() if msg else "")
        self.r = len(relations)
        self.n = L.figaro_plan_num_cols(self._handle)
        self.ncols = [int(rel.ncols) for rel in relations]

    @classmethod
    def tuned(cls, relations: Sequence, values: Sequence, candidates=None, reps: int = 3, stream=None):
        """Autotuned plan: builds the plan under several option sets (tile
        variant, wave cap), times the forward pass of each on `values`
        (caller order, (n_i, m_i) float64 device tensors) and keeps the
        fastest.  `candidates`: list of dicts with keys tile_items,
        waves_per_task, variant (None: the library's default set)."""
        import torch
        L = lib()
        descs, keep = _device_descs(relations)
        r = len(relations)
        ptrs = (ctypes.c_void_p * r)()
        lds = (ctypes.c_int64 * r)()
        for i, v in enumerate(values):
            if v.dtype != torch.float64 or not v.is_cuda or v.stride(1) != 1:
                raise ValueError("values must be float64 device tensors of shape (n_i, m_i), rows contiguous")
            ptrs[i] = v.data_ptr()
            lds[i] = max(v.stride(0), v.shape[1], 1)
        if candidates:
            cand = (PlanOptions * len(candidates))()
            for k, c in enumerate(candidates):
                cand[k] = PlanOptions(int(c.get("tile_items", 0)), int(c.get("waves_per_task", 0)), 0,
                                      int(c.get("variant", 0)), 0)
            nc = len(candidates)
        else:
            cand, nc = None, 0
        h = ctypes.c_void_p()
        st = L.figaro_plan_create_tuned(ctypes.byref(h), r, descs, ptrs, lds, nc, cand, reps,
                                        _stream_handle(stream))
        del keep
        if st != FIGARO_OK:
            msg = L.figaro_last_error(None)
            raise FigaroError(st, msg.decode() if msg else "")
        return cls(relations, _handle=h)

    def tuning(self):
        """(chosen options as a dict, milliseconds per forward pass) of a
        plan built by Plan.tuned()."""
        o = PlanOptions()
        ms = ctypes.c_double()
        _check(lib().figaro_plan_tuning(self._handle, ctypes.byref(o), ctypes.byref(ms)), self._handle)
        return {"tile_items": o.tile_items, "waves_per_task": o.waves_per_task, "variant": o.variant}, ms.value

    def _init_host(self, relations, tile_items, waves_per_task):
        """Keys given as host arrays; only the key analysis runs (validation,
        reduction, order, count queries).  Needs no GPU."""
        L = lib()
        self._handle = ctypes.c_void_p()
        r = len(relations)
        descs = (RelationDesc * r)()
        keep = []
        for i, rel in enumerate(relations):
            attrs = np.ascontiguousarray(np.asarray(rel.key_attrs, dtype=np.int32))
            keys = np.ascontiguousarray(np.asarray(rel.keys))
            if keys.dtype not in (np.int32, np.int64):
                keys = keys.astype(np.int64)
            keep += [attrs, keys]
            descs[i].rows = int(rel.values.shape[1]) if hasattr(rel, "values") else int(keys.shape[1])
            descs[i].num_keys = len(rel.key_attrs)
            descs[i].key_attr = attrs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            descs[i].key_cols = ctypes.c_void_p(keys.ctypes.data if keys.size else 0)
            descs[i].key_dtype = 8 if keys.dtype == np.int64 else 4
            descs[i].num_cols = int(rel.values.shape[0]) if hasattr(rel, "values") else int(rel.ncols)
            descs[i].parent = int(rel.parent)
        opts = PlanOptions(tile_items, waves_per_task, 1, 0, 1)
        st = L.figaro_plan_create(ctypes.byref(self._handle), r, descs, ctypes.byref(opts), None)
        if st != FIGARO_OK:
            msg = L.figaro_last_error(None)
            raise FigaroError(st, msg.decode() if msg else "")
        self.r = r
        self.n = L.figaro_plan_num_cols(self._handle)
        self.ncols = [int(descs[i].num_cols) for i in range(r)]

    # -- info ---------------------------------------------------------------
    def rows(self, i: int) -> int:
        return int(lib().figaro_plan_rows(self._handle, i))

    def input_rows(self, i: int) -> int:
        return int(lib().figaro_plan_input_rows(self._handle, i))

    def dropped_rows(self, i: int) -> int:
        return int(lib().figaro_plan_dropped_rows(self._handle, i))

    @property
    def join_rows(self) -> float:
        return float(lib().figaro_plan_join_rows(self._handle))

    @property
    def workspace_bytes(self) -> int:
        return int(lib().figaro_plan_workspace_bytes(self._handle))

    def permutation(self, i: int) -> np.ndarray:
        out = np.zeros(self.input_rows(i), dtype=np.int64)
        _check(lib().figaro_plan_permutation(self._handle, i,
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               self._handle)
        return out

    def num_groups(self, i: int, which: int = 0) -> int:
        return int(lib().figaro_plan_num_groups(self._handle, i, which))

    def group_first_rows(self, i: int, which: int = 0) -> np.ndarray:
        out = np.zeros(max(self.num_groups(i, which), 0), dtype=np.int64)
        _check(lib().figaro_plan_group_first_rows(self._handle, i, which,
                                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               self._handle)
        return out

    def counts(self, i: int, kind: str) -> np.ndarray:
        which = 1 if kind in ("phi_up", "phi_down") else 0
        out = np.zeros(max(self.num_groups(i, which), 0), dtype=np.int64)
        _check(lib().figaro_plan_counts(self._handle, i, COUNT_KINDS[kind],
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               self._handle)
        return out

    # -- data movement ------------------------------------------------------
    def to_plan_order(self, i: int, values, stream=None):
        """(n_i, m_i) caller-order device tensor -> (n_i, kept rows) plan order.
        The rows of the result are padded to a multiple of 16 doubles, so every
        column starts 128-byte aligned (the head/tail kernels then stage full
        tiles with 16-byte copies)."""
        import torch
        assert values.dtype == torch.float64 and values.is_cuda and values.stride(1) == 1
        rows = self.rows(i)
        ld = max((rows + 15) // 16 * 16, 16)
        out = torch.empty((values.shape[0], ld), dtype=torch.float64, device=values.device)[:, :rows]
        _check(lib().figaro_permute_values(self._handle, i, ctypes.c_void_p(values.data_ptr()),
                                           values.stride(0), ctypes.c_void_p(out.data_ptr()),
                                           max(out.stride(0), 1), _stream_handle(stream)), self._handle)
        return out

    def from_plan_order(self, i: int, values, stream=None):
        """(n_i, kept rows) plan-order tensor -> (n_i, m_i) caller order, zeros
        for rows removed by the reduction."""
        import torch
        out = torch.empty((values.shape[0], self.input_rows(i)), dtype=torch.float64, device=values.device)
        _check(lib().figaro_unpermute_values(self._handle, i, ctypes.c_void_p(values.data_ptr()),
                                             max(values.stride(0), 1), ctypes.c_void_p(out.data_ptr()),
                                             max(out.stride(0), 1), _stream_handle(stream)), self._handle)
        return out

    def _value_args(self, values):
        import torch
        if len(values) != self.r:
            raise ValueError("one value tensor per relation")
        ptrs = (ctypes.c_void_p * self.r)()
        lds = (ctypes.c_int64 * self.r)()
        for i, v in enumerate(values):
            if v.dtype != torch.float64 or not v.is_cuda or v.stride(1) != 1:
                raise ValueError("values must be float64 device tensors of shape (n_i, rows), rows contiguous")
            if v.shape[0] != self.ncols[i] or v.shape[1] < self.rows(i):
                raise ValueError(f"values[{i}] has shape {tuple(v.shape)}")
            ptrs[i] = v.data_ptr()
            lds[i] = max(v.stride(0), self.rows(i))
        return ptrs, lds

    # -- compute ------------------------------------------------------------
    def r_factor(self, values: List, out=None, stream=None):
        """R (n x n, upper triangular, non-negative diagonal) of the join."""
        import torch
        ptrs, lds = self._value_args(values)
        if out is None:
            out = torch.empty((self.n, self.n), dtype=torch.float64, device=values[0].device)
        # column-major n x n == row-major transpose: allocate (n, n) and read .T
        _check(lib().figaro_r(self._handle, ptrs, lds, ctypes.c_void_p(out.data_ptr()),
                              _stream_handle(stream)), self._handle)
        return out.T

    def join_multiply(self, values: List, M, col_scale=None, row0: int = 0, nrows=None, with_ids: bool = False,
                      stream=None):
        """Rows row0 .. row0 + nrows - 1 of A M for the join matrix A (never
        materialised) and an n x k device matrix M, columns scaled by
        col_scale; with with_ids also the caller row index of every
        relation's tuple in each row ((r, nrows) int64).  Returns the
        (nrows, k) rows (and the ids)."""
        import torch
        ptrs, lds = self._value_args(values)
        if nrows is None:
            nrows = int(self.join_rows) - row0
        k = int(M.shape[1])
        Mc = M.detach().to(torch.float64).T.contiguous()      # column-major n x k
        dev = values[0].device
        nbytes = int(lib().figaro_join_multiply_workspace_bytes(self._handle, k))
        work = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=dev)
        out = torch.empty((k, max(nrows, 1)), dtype=torch.float64, device=dev)
        ids = torch.empty((self.r, max(nrows, 1)), dtype=torch.int64, device=dev) if with_ids else None
        sc = col_scale.detach().to(torch.float64).contiguous() if col_scale is not None else None
        _check(lib().figaro_join_multiply(self._handle, ptrs, lds, ctypes.c_void_p(Mc.data_ptr()), self.n, k,
                                          ctypes.c_void_p(sc.data_ptr()) if sc is not None else None, row0, nrows,
                                          ctypes.c_void_p(out.data_ptr()), max(nrows, 1),
                                          ctypes.c_void_p(ids.data_ptr()) if ids is not None else None,
                                          max(nrows, 1), ctypes.c_void_p(work.data_ptr()), work.numel() * 8,
                                          _stream_handle(stream)), self._handle)
        rows = out[:, :nrows].T
        return (rows, ids[:, :nrows]) if with_ids else rows

    def r_backward(self, values: List, R, dR, stream=None):
        """Gradients of a loss with respect to the values (plan order), given
        R from r_factor() and dR = dLoss/dR (only its upper triangle is used)."""
        import torch
        ptrs, lds = self._value_args(values)
        Rc = R.detach().T.contiguous()     # column-major n x n
        dRc = dR.detach().to(torch.float64).T.contiguous()
        outs = [torch.empty((self.ncols[i], max(self.rows(i), 1)), dtype=torch.float64, device=values[0].device)
                for i in range(self.r)]
        optr = (ctypes.c_void_p * self.r)(*[o.data_ptr() for o in outs])
        olds = (ctypes.c_int64 * self.r)(*[max(o.stride(0), self.rows(i)) for i, o in enumerate(outs)])
        _check(lib().figaro_r_backward(self._handle, ptrs, lds, ctypes.c_void_p(Rc.data_ptr()),
                                       ctypes.c_void_p(dRc.data_ptr()), optr, olds, _stream_handle(stream)),
               self._handle)
        return [o[:, :self.rows(i)] for i, o in enumerate(outs)]

    def backward_status(self, stream=None) -> str:
        st = lib().figaro_backward_status(self._handle, _stream_handle(stream))
        return STATUS_NAMES.get(st, str(st))

    def r0(self, values: List, stream=None):
        """The intermediate R0 (rows x n) and the block id of every row."""
        import torch
        ptrs, lds = self._value_args(values)
        rows = int(lib().figaro_r0_rows(self._handle))
        buf = torch.empty((self.n, max(rows, 1)), dtype=torch.float64, device=values[0].device)
        blk = torch.empty((max(rows, 1),), dtype=torch.int32, device=values[0].device)
        _check(lib().figaro_r0(self._handle, ptrs, lds, ctypes.c_void_p(buf.data_ptr()), max(rows, 1),
                               ctypes.c_void_p(blk.data_ptr()), _stream_handle(stream)), self._handle)
        return buf[:, :rows].T, blk[:rows]

    def debug_stack(self, values, stream=None):
        """Partial R factors and root rows before the post-processing TSQR."""
        ptrs, lds = self._value_args(values)
        rows = int(lib().figaro_debug_stack_rows(self._handle))
        out = np.zeros((self.n, max(rows, 1)), dtype=np.float64)
        _check(lib().figaro_debug_stack(self._handle, ptrs, lds, ctypes.c_void_p(out.ctypes.data),
                                        _stream_handle(stream)), self._handle)
        return out[:, :rows].T

    def debug_stack_layout(self):
        out = np.zeros(3 * 256, dtype=np.int64)
        k = lib().figaro_debug_stack_layout(self._handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 256)
        return out[:3 * k].reshape(k, 3)

    # -- profiling ------------------------------------------------------------
    PROFILE_CLASSES = {0: "heads_tails", 1: "project_away", 2: "upper_levels", 3: "join",
                       4: "root", 5: "post_tsqr", 6: "backward"}

    def profile_enable(self, capacity: int = 4096):
        _check(lib().figaro_profile_enable(self._handle, capacity), self._handle)

    def profile_reset(self):
        _check(lib().figaro_profile_reset(self._handle), self._handle)

    def profile_read(self):
        """{class name: (total ms, launches, algorithmic bytes, flops)}"""
        out = {}
        for k, name in self.PROFILE_CLASSES.items():
            ms, n, b, f = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            _check(lib().figaro_profile_read(self._handle, k, ctypes.byref(ms), ctypes.byref(n),
                                             ctypes.byref(b), ctypes.byref(f)), self._handle)
            out[name] = (ms.value, n.value, b.value, f.value)
        return out

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            lib().figaro_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_autograd():
    import torch

    class FigaroR(torch.autograd.Function):
        """R of the join as a differentiable function of the relation values
        (plan order).  Backward runs the library's adjoint."""

        @staticmethod
        def forward(ctx, plan, *values):
            R = plan.r_factor(list(values)).clone()
            ctx.plan = plan
            ctx.save_for_backward(R, *values)
            return R

        @staticmethod
        def backward(ctx, dR):
            R, *values = ctx.saved_tensors
            grads = ctx.plan.r_backward(list(values), R, dR.contiguous())
            return (None, *grads)

    return FigaroR


_FigaroR = None


def figaro_r(plan, *values):
    """Differentiable R (torch.autograd): figaro_r(plan, v_0, ..., v_{r-1})."""
    global _FigaroR
    if _FigaroR is None:
        _FigaroR = _make_autograd()
    return _FigaroR.apply(plan, *values)


class _RelView:
    def __init__(self, key_attrs, keys, ncols, parent):
        self.key_attrs = key_attrs
        self.keys = keys
        self.ncols = ncols
        self.parent = parent


def shape_class(relations) -> str:
    """Tuning class of an instance: its total column count in the buckets of
    the register tiles (8, 16, 32, 40, wider) and its tuple count in half
    decades.  Instances of one class share the autotuner's choice."""
    import math
    n = sum(int(r.ncols) for r in relations)
    m = sum(int(r.keys.shape[-1]) for r in relations)
    nb = next((b for b in (8, 16, 32, 40) if n <= b), "wide")
    return f"n{nb}_m{math.floor(2 * math.log10(max(m, 1))) / 2:.1f}"


class TuningCache:
    """The option set the autotuner (Plan.tuned) picks for each shape class,
    tuned on the first instance of the class that asks and kept in a JSON
    file (path None: in memory only)."""

    def __init__(self, path=None):
        import json
        self.path = path
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def options(self, relations, values, reps: int = 2) -> dict:
        """Options (tile_items, waves_per_task, variant) for an instance:
        from the cache, or by tuning it (values: caller order, as for
        Plan.tuned)."""
        key = shape_class(relations)
        if key not in self.entries:
            p = Plan.tuned(relations, values, reps=reps)
            opts, ms = p.tuning()
            p.close()
            self.entries[key] = dict(opts, ms=ms)
        e = self.entries[key]
        return {k: int(e[k]) for k in ("tile_items", "waves_per_task", "variant")}

    def save(self):
        import json
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)


def instance_views(inst, device="cuda") -> List:
    """Relation views (keys on the device) of a synth.Instance-like object."""
    import torch
    rels = []
    for rel in inst.rels:
        keys = torch.as_tensor(np.ascontiguousarray(rel.keys)).to(device)
        if keys.dim() == 1:
            keys = keys[None, :]
        rels.append(_RelView(list(rel.key_attrs), keys, rel.values.shape[0], rel.parent))
    return rels


def plan_from_instance(inst, device="cuda", **kw) -> Plan:
    """Plan for a synth.Instance-like object (keys moved to the device)."""
    return Plan(instance_views(inst, device), **kw)


def device_values(plan: Plan, inst, device="cuda") -> List:
    """Caller-order values of an instance -> plan-order device tensors."""
    import torch
    out = []
    for i, rel in enumerate(inst.rels):
        v = torch.as_tensor(np.ascontiguousarray(rel.values, dtype=np.float64)).to(device)
        out.append(plan.to_plan_order(i, v))
    return out


def _host_descs(inst, parents=None):
    """Relation descriptors with host int64 keys for the join-tree calls."""
    keep = []
    arr = (RelationDesc * inst.r)()
    for i, rel in enumerate(inst.rels):
        attrs = np.ascontiguousarray(rel.key_attrs, dtype=np.int32)
        keys = np.ascontiguousarray(rel.keys, dtype=np.int64).reshape(len(rel.key_attrs), rel.rows)
        keep += [attrs, keys]
        arr[i].rows = rel.rows
        arr[i].num_keys = len(rel.key_attrs)
        arr[i].key_attr = attrs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        arr[i].key_cols = ctypes.c_void_p(keys.ctypes.data)
        arr[i].key_dtype = 8
        arr[i].num_cols = rel.ncols
        arr[i].parent = rel.parent if parents is None else int(parents[i])
    return arr, keep


def join_tree_cost(inst, parents=None) -> float:
    """Score (QR work: rows x columns^2 over the blocks of R0) of the join
    tree given by the instance's parents (or `parents`)."""
    arr, keep = _host_descs(inst, parents)
    c = ctypes.c_double()
    _check(lib().figaro_join_tree_cost(inst.r, arr, 1, ctypes.byref(c), None), None)
    return c.value


def choose_join_tree(inst):
    """The join tree (parent of every relation, -1 for the root) with the
    lowest score over all join trees and roots, and that score."""
    arr, keep = _host_descs(inst)
    parents = (ctypes.c_int32 * inst.r)()
    c = ctypes.c_double()
    _check(lib().figaro_choose_join_tree(inst.r, arr, 1, parents, ctypes.byref(c), None), None)
    return [int(x) for x in parents], c.value


def debug_tile_rows(n: int, variant: int = 0) -> int:
    """Rows per register tile of one wave of the dense TSQR kernel."""
    return int(lib().figaro_debug_tile_rows(n, variant))


def debug_dense_rows(n: int, variant: int, tiles_per_wave: int) -> int:
    """Rows that one workgroup of the dense TSQR kernel folds."""
    return int(lib().figaro_debug_dense_rows(n, variant, tiles_per_wave))


def debug_dense_step(A, workgroups: int, tiles_per_wave: int, variant: int = 0, stream=None):
    """One launch of the dense TSQR kernel on a device FP64 matrix A (rows x
    n, column-major, i.e. A.T contiguous).  Returns the n x n sign-normalised
    R for one workgroup, else the (workgroups*n) x n stack of per-workgroup R."""
    import torch
    rows, n = A.shape
    At = A.t().contiguous() if not A.t().is_contiguous() else A.t()
    if workgroups == 1:
        R = torch.zeros((n, n), dtype=torch.float64, device=A.device)
        _check(lib().figaro_debug_dense_step(n, rows, ctypes.c_void_p(At.data_ptr()), max(rows, 1), 1,
                                             tiles_per_wave, variant, None, 0, ctypes.c_void_p(R.data_ptr()),
                                             _stream_handle(stream)), None)
        return R.t()
    out = torch.zeros((n, workgroups * n), dtype=torch.float64, device=A.device)
    _check(lib().figaro_debug_dense_step(n, rows, ctypes.c_void_p(At.data_ptr()), max(rows, 1), workgroups,
                                         tiles_per_wave, variant, ctypes.c_void_p(out.data_ptr()), workgroups * n,
                                         None, _stream_handle(stream)), None)
    return out.t()


def svd_of_r(R, stream=None):
    """sigma (decreasing), U_R and V of an n x n device matrix R (the R of a
    join: sigma and V are then the join matrix's singular values and right
    singular vectors)."""
    import torch
    n = int(R.shape[0])
    Rc = R.detach().T.contiguous()
    dev = R.device
    sigma = torch.empty(n, dtype=torch.float64, device=dev)
    U = torch.empty((n, n), dtype=torch.float64, device=dev)
    V = torch.empty((n, n), dtype=torch.float64, device=dev)
    work = torch.empty(2 * n * n, dtype=torch.float64, device=dev)
    _check(lib().figaro_svd_r(n, ctypes.c_void_p(Rc.data_ptr()), ctypes.c_void_p(sigma.data_ptr()),
                              ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                              ctypes.c_void_p(work.data_ptr()), _stream_handle(stream)), None)
    return sigma, U.T, V.T


def r_inverse(R, stream=None):
    """R^-1 of an upper-triangular n x n device matrix."""
    import torch
    n = int(R.shape[0])
    Rc = R.detach().T.contiguous()
    X = torch.empty((n, n), dtype=torch.float64, device=R.device)
    _check(lib().figaro_r_inverse(n, ctypes.c_void_p(Rc.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                  _stream_handle(stream)), None)
    return X.T


def _colmajor(A):
    """(rows, n) device tensor -> (tensor holding column-major storage,
    leading dimension): A itself when its rows are contiguous and its columns
    at least `rows` apart, else a column-major copy."""
    rows, n = A.shape
    if A.stride(0) == 1 and (n <= 1 or A.stride(1) >= max(rows, 1)):
        return A, max(A.stride(1) if n > 1 else rows, 1)
    return A.t().contiguous(), max(rows, 1)


def tsqr_workspace_bytes(rows: int, n: int) -> int:
    return int(lib().figaro_tsqr_workspace_bytes(rows, n))


def tsqr(A, workspace=None, stream=None):
    """R (n x n, non-negative diagonal) of a device FP64 matrix A (rows x n)
    by the post-processing TSQR; the partial R's go to `workspace` (a device
    tensor of at least tsqr_workspace_bytes(rows, n) bytes), allocated here
    when it is None."""
    import torch
    rows, n = A.shape
    At, lda = _colmajor(A)
    R = torch.empty((n, n), dtype=torch.float64, device=A.device)
    if workspace is None:
        nbytes = tsqr_workspace_bytes(rows, n)
        workspace = torch.empty((max(nbytes, 8) + 7) // 8, dtype=torch.float64, device=A.device)
    _check(lib().figaro_tsqr(rows, n, ctypes.c_void_p(At.data_ptr()), lda, ctypes.c_void_p(R.data_ptr()),
                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                             _stream_handle(stream)), None)
    return R.t()


def tsqr_noalloc(A, R=None, stream=None):
    """figaro_tsqr_noalloc(): as tsqr(), with the library's static device
    array instead of a workspace.  A must already be column-major (rows
    contiguous), since a copy would allocate; R (n x n, column-major storage)
    may be passed in to keep the call free of allocations."""
    import torch
    rows, n = A.shape
    if not (A.stride(0) == 1 and (n <= 1 or A.stride(1) >= max(rows, 1))):
        raise ValueError("tsqr_noalloc needs a column-major A")
    lda = max(A.stride(1) if n > 1 else rows, 1)
    if R is None:
        R = torch.empty((n, n), dtype=torch.float64, device=A.device).t()
    elif R.shape != (n, n) or R.stride() != (1, n) or R.dtype != torch.float64:
        raise ValueError("R must be an n x n column-major FP64 tensor")
    _check(lib().figaro_tsqr_noalloc(rows, n, ctypes.c_void_p(A.data_ptr()), lda, ctypes.c_void_p(R.data_ptr()),
                                     _stream_handle(stream)), None)
    return R


class Batch:
    """Many independent instances (one plan each) per call: instances run
    side by side on the batch's streams, forked from and joined back to the
    caller's stream.  capture()/launch() record the whole forward batch once
    as a HIP graph and replay it."""

    def __init__(self, plans: Sequence[Plan], streams: int = 0):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._handle.value for p in self.plans])
        self._handle = ctypes.c_void_p()
        st = lib().figaro_batch_create(ctypes.byref(self._handle), len(self.plans), arr, streams)
        if st != FIGARO_OK:
            msg = lib().figaro_last_error(None)
            raise FigaroError(st, msg.decode() if msg else "")

    def stream_of(self, i: int) -> int:
        return int(lib().figaro_batch_stream_of(self._handle, i))

    def _marshal(self, values_list):
        keep, vptrs, lptrs = [], [], []
        for p, vals in zip(self.plans, values_list):
            ptrs, lds = p._value_args(vals)
            keep += [ptrs, lds]
            vptrs.append(ctypes.cast(ptrs, ctypes.POINTER(ctypes.c_void_p)))
            lptrs.append(ctypes.cast(lds, ctypes.POINTER(ctypes.c_int64)))
        V = (ctypes.POINTER(ctypes.c_void_p) * len(self.plans))(*vptrs)
        LD = (ctypes.POINTER(ctypes.c_int64) * len(self.plans))(*lptrs)
        keep += [V, LD]
        return V, LD, keep

    def _outs(self, values_list, outs):
        import torch
        if outs is None:
            outs = [torch.empty((p.n, p.n), dtype=torch.float64, device=v[0].device)
                    for p, v in zip(self.plans, values_list)]
        R = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        return outs, R

    def r(self, values_list, outs=None, stream=None):
        """R of every instance (list of n_i x n_i tensors)."""
        V, LD, keep = self._marshal(values_list)
        outs, R = self._outs(values_list, outs)
        _check(lib().figaro_r_batched(self._handle, V, LD, R, _stream_handle(stream)), None)
        return [o.T for o in outs]

    def r_backward(self, values_list, Rs, dRs, stream=None):
        """Gradients of every instance (list of per-relation lists, plan order)."""
        import torch
        V, LD, keep = self._marshal(values_list)
        Rc = [R.detach().T.contiguous() for R in Rs]
        dRc = [d.detach().to(torch.float64).T.contiguous() for d in dRs]
        Rp = (ctypes.c_void_p * len(Rc))(*[x.data_ptr() for x in Rc])
        dRp = (ctypes.c_void_p * len(dRc))(*[x.data_ptr() for x in dRc])
        grads, gp, gl = [], [], []
        for p, vals in zip(self.plans, values_list):
            g = [torch.empty((p.ncols[i], max(p.rows(i), 1)), dtype=torch.float64, device=vals[0].device)
                 for i in range(p.r)]
            grads.append(g)
            a = (ctypes.c_void_p * p.r)(*[x.data_ptr() for x in g])
            l = (ctypes.c_int64 * p.r)(*[max(x.stride(0), p.rows(i)) for i, x in enumerate(g)])
            keep += [a, l]
            gp.append(ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p)))
            gl.append(ctypes.cast(l, ctypes.POINTER(ctypes.c_int64)))
        GP = (ctypes.POINTER(ctypes.c_void_p) * len(gp))(*gp)
        GL = (ctypes.POINTER(ctypes.c_int64) * len(gl))(*gl)
        _check(lib().figaro_r_backward_batched(self._handle, V, LD, Rp, dRp, GP, GL, _stream_handle(stream)),
               None)
        return [[x[:, :p.rows(i)] for i, x in enumerate(g)] for p, g in zip(self.plans, grads)]

    def capture(self, values_list, outs, stream):
        """Capture the forward batch on these buffers into a HIP graph; `outs`
        are the n_i x n_i output tensors (written on every launch)."""
        V, LD, keep = self._marshal(values_list)
        outs, R = self._outs(values_list, outs)
        _check(lib().figaro_batch_capture(self._handle, V, LD, R, _stream_handle(stream)), None)
        self._captured = (values_list, outs, keep)
        return [o.T for o in outs]

    def launch(self, stream=None):
        _check(lib().figaro_batch_launch(self._handle, _stream_handle(stream)), None)

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            lib().figaro_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
