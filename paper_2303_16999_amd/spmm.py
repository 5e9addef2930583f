"""ctypes binding of libspmm.so (the C ABI in include/spmm.h).

Argument marshalling only: every step of the SpMM runs in the library's HIP
kernels. torch tensors supply device memory and streams; their data pointers
are passed straight through. There is no fallback: if the library is missing,
`lib()` raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspmm.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_CAPACITY, ERR_BAD_INDEX, ERR_OOM, ERR_HIP, ERR_REJECTED = range(8)
F32, F16, BF16, FP8_E4M3 = range(4)
DTYPE_CODES = {"f32": F32, "f16": F16, "bf16": BF16, "fp8": FP8_E4M3}

# every symbol the header declares, with its ctypes signature
_c_i64, _c_i32, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
_pi32, _pi64 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)


class PlanOpts(ctypes.Structure):
    _fields_ = [("group_rows", ctypes.c_int32), ("num_panels", ctypes.c_int32),
                ("n_hint", ctypes.c_int32), ("variant", ctypes.c_int32), ("dense_dispatch", ctypes.c_int32)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("manual", ctypes.c_int32), ("simulate", ctypes.c_int32), ("max_tokens", ctypes.c_int64)]


class ServeDone(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("n", ctypes.c_int64), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("requests_done", ctypes.c_int64), ("tokens_done", ctypes.c_int64),
                ("problems_run", ctypes.c_int64), ("peak_pool_bytes", ctypes.c_int64),
                ("peak_active", ctypes.c_int32), ("pending", ctypes.c_int32), ("active", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("busy_s", ctypes.c_double)]


SERVE_CONTINUOUS, SERVE_PLAIN = 0, 1

SIGNATURES = {
    "spmm_last_error": ([], ctypes.c_char_p),
    "spmm_plan_static": ([_c_i64, _c_i64, _c_i32, _vp, _c_i32, _c_i32, _c_i32, ctypes.POINTER(PlanOpts),
                          ctypes.POINTER(_vp)], _c_i32),
    "spmm_plan_set_values": ([_vp, _vp, _vp, _vp], _c_i32),
    "spmm_run_static": ([_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp], _c_i32),
    "spmm_plan_info": ([_vp, _pi64, _pi32, _pi32, _pi32, _pi32], _c_i32),
    "spmm_plan_export": ([_vp, _vp, _vp, _vp, _vp], _c_i32),
    "spmm_plan_destroy": ([_vp], _c_i32),
    "spmm_dynamic_create": ([_c_i64, _c_i64, _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, ctypes.POINTER(PlanOpts),
                             ctypes.POINTER(_vp)], _c_i32),
    "spmm_run_dynamic": ([_vp, _vp, _vp, _vp, _vp, _vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _vp], _c_i32),
    "spmm_dynamic_export": ([_vp, _vp, _vp, _vp, _vp, _pi64], _c_i32),
    "spmm_dynamic_info": ([_vp, _pi32, _pi32, _pi32], _c_i32),
    "spmm_dynamic_destroy": ([_vp], _c_i32),
    "spmm_run_dynamic_noalloc": ([_c_i64, _c_i64, _c_i32, _c_i64, _c_i32, _c_i32, _c_i32, _vp, _vp, _vp, _vp, _vp,
                                  _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _vp], _c_i32),
    "spmm_autotune_static": ([_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _pi32, ctypes.POINTER(ctypes.c_float)],
                             _c_i32),
    "spmm_autotune_static_all": ([_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _c_i32, _pi32,
                                  ctypes.POINTER(ctypes.c_float), _pi32, _pi32], _c_i32),
    "spmm_plan_variant": ([_vp, _c_i64, _pi32], _c_i32),
    "spmm_autotune_clear": ([], _c_i32),
    "spmm_plan_dispatch": ([_vp, ctypes.POINTER(ctypes.c_double), _pi32], _c_i32),
    "spmm_plan_memory": ([_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _c_i32),
    "spmm_group_create": ([_c_i32, ctypes.POINTER(_vp)], _c_i32),
    "spmm_group_run": ([_vp, _c_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _c_i32),
    "spmm_group_destroy": ([_vp], _c_i32),
    "spmm_serve_create": ([_vp, _c_i32, _vp, _vp, ctypes.POINTER(ServeOpts), ctypes.POINTER(_vp)], _c_i32),
    "spmm_serve_submit": ([_vp, ctypes.c_uint64, _c_i64, _vp, _vp, _c_i64], _c_i32),
    "spmm_serve_poll": ([_vp, ctypes.POINTER(ServeDone), _c_i32, _pi32], _c_i32),
    "spmm_serve_step": ([_vp, _pi32], _c_i32),
    "spmm_serve_drain": ([_vp], _c_i32),
    "spmm_serve_stats": ([_vp, ctypes.POINTER(ServeStats)], _c_i32),
    "spmm_serve_destroy": ([_vp], _c_i32),
    "spmm_serve_clock": ([], ctypes.c_double),
    "spmm_plan_transpose": ([_vp, ctypes.POINTER(PlanOpts), ctypes.POINTER(_vp)], _c_i32),
    "spmm_plan_ell": ([_c_i64, _c_i64, _c_i32, _c_i32, _vp, _c_i32, _c_i32, _c_i32, ctypes.POINTER(PlanOpts),
                       ctypes.POINTER(_vp)], _c_i32),
    "spmm_plan_set_values_ell": ([_vp, _vp, _vp, _vp], _c_i32),
    "spmm_speedup_model": ([_c_i64, ctypes.c_double, _c_i32, ctypes.POINTER(ctypes.c_double)], _c_i32),
    "spmm_sddmm": ([_vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _vp], _c_i32),
}

_LIB = None


class SpmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("spmm status %d: %s" % (status, message))
        self.status = status


def lib():
    """Load libspmm.so (built by paper_2303_16999_amd.build); raise if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libspmm.so is not built; run `python -m paper_2303_16999_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def check(status):
    if status != OK:
        raise SpmmError(status, lib().spmm_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


_TORCH = None


def _torch():
    """torch, imported on first use (the module itself does not need it)."""
    global _TORCH
    if _TORCH is None:
        import torch
        _TORCH = torch
    return _TORCH


def _stream(stream):
    if stream is None:
        torch = _torch()
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)  # the handle, without a Stream object
        if raw is not None:
            return raw(torch.cuda.current_device())
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _opts(group_rows=0, num_panels=0, n_hint=0, variant=0, dense_dispatch=0):
    return PlanOpts(int(group_rows), int(num_panels), int(n_hint), int(variant), int(dense_dispatch))


_TORCH_DTYPES = None


def torch_dtype(code):
    global _TORCH_DTYPES
    if _TORCH_DTYPES is None:
        torch = _torch()
        _TORCH_DTYPES = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16, FP8_E4M3: torch.uint8}
    return _TORCH_DTYPES[code]


_ELEM_BYTES = {F32: 4, F16: 2, BF16: 2, FP8_E4M3: 1}


def check_dense(t, rows, n, code, name, on_gpu=True):
    """Rejects a dense operand (X or Y) that the kernels would read or write
    past its end: a 2-D torch tensor of the plan's dtype with unit column
    stride, at least `rows` rows and n columns, on the GPU (on_gpu=False
    leaves that last check to the caller). Only shapes, strides, dtypes and
    the device are looked at."""
    if not isinstance(t, _torch().Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dim() != 2:
        raise ValueError("%s must be 2-D, got %d dimensions" % (name, t.dim()))
    if t.dtype != torch_dtype(code):
        raise ValueError("%s has dtype %s, the plan needs %s" % (name, t.dtype, torch_dtype(code)))
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("%s must have unit column stride" % name)
    if t.shape[0] < rows:
        raise ValueError("%s has %d rows, the plan needs %d" % (name, t.shape[0], rows))
    if n < 0 or n > t.shape[1]:
        raise ValueError("n = %d does not fit the %d columns of %s" % (n, t.shape[1], name))
    if on_gpu:
        check_gpu(t, name)


def check_gpu(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)


def check_flat(t, count, elem_bytes, name, dtype=None, on_gpu=True):
    """Rejects a device buffer of fewer than `count` elements of `elem_bytes`
    bytes (values, scales, indices), of the wrong dtype, or not on the GPU."""
    if not isinstance(t, _torch().Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if dtype is not None:
        if t.dtype != dtype:
            raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    elif t.element_size() != elem_bytes:
        raise ValueError("%s has %d-byte elements, expected %d" % (name, t.element_size(), elem_bytes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < count:
        raise ValueError("%s holds %d elements, %d are needed" % (name, t.numel(), count))
    if on_gpu:
        check_gpu(t, name)


def _ncols(t):
    """Columns of a 2-D operand (0 for anything else, which the checks reject)."""
    shape = getattr(t, "shape", ())
    return int(shape[1]) if len(shape) == 2 else 0


def _ld(t, ld, name):
    if ld is None:
        return int(t.stride(0))
    if int(ld) != int(t.stride(0)):
        raise ValueError("leading dimension of %s must be its row stride %d" % (name, t.stride(0)))
    return int(ld)


def autotune_clear():
    """spmm_autotune_clear: forget the process-wide table of tuned variants."""
    check(lib().spmm_autotune_clear())


class StaticPlan:
    """spmm_plan_static / spmm_plan_set_values / spmm_run_static."""

    def __init__(self, m, k, b, block_mask, w="f16", x=None, y=None, group_rows=0, num_panels=0, n_hint=0,
                 variant=0, dense_dispatch=0):
        x = x or ("f16" if w == "fp8" else w)
        y = y or x
        mask = np.ascontiguousarray(np.asarray(block_mask, dtype=np.uint8))
        if b > 0 and mask.size != (-(-int(m) // int(b))) * (-(-int(k) // int(b))):
            raise ValueError("block_mask must have ceil(m/b) x ceil(k/b) entries")
        self.m, self.k, self.b = int(m), int(k), int(b)
        self.w, self.x, self.y = DTYPE_CODES[w], DTYPE_CODES[x], DTYPE_CODES[y]
        h = _vp()
        opts = _opts(group_rows, num_panels, n_hint, variant, dense_dispatch)
        check(lib().spmm_plan_static(self.m, self.k, self.b, mask.ctypes.data_as(_vp), self.w, self.x, self.y,
                                     ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.mb, self.kb = -(-self.m // self.b), -(-self.k // self.b)

    def info(self):
        nnz, gr, ng, npn, nh = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().spmm_plan_info(self._h, ctypes.byref(nnz), ctypes.byref(gr), ctypes.byref(ng), ctypes.byref(npn),
                                   ctypes.byref(nh)))
        return {"nnzb": nnz.value, "group_rows": gr.value, "num_groups": ng.value, "num_panels": npn.value,
                "num_split_rows": nh.value}

    def memory(self):
        """spmm_plan_memory: (device bytes of all the plan's buffers, bytes of its one value copy)."""
        db, vb = ctypes.c_int64(), ctypes.c_int64()
        check(lib().spmm_plan_memory(self._h, ctypes.byref(db), ctypes.byref(vb)))
        return db.value, vb.value

    def dispatch(self):
        """spmm_plan_dispatch: (speedup model's sparse/dense ratio, keeps a dense copy)."""
        pr, hd = ctypes.c_double(), ctypes.c_int32()
        check(lib().spmm_plan_dispatch(self._h, ctypes.byref(pr), ctypes.byref(hd)))
        return pr.value, bool(hd.value)

    def _nnzb(self):
        if getattr(self, "_nnzb_cache", None) is None:
            self._nnzb_cache = self.info()["nnzb"]
        return self._nnzb_cache

    def set_values(self, values, scales=None, stream=None):
        import torch
        nnzb = self._nnzb()
        if nnzb:
            check_flat(values, nnzb * self.b * self.b, _ELEM_BYTES[self.w], "values", on_gpu=False)
            if scales is not None:
                check_flat(scales, nnzb, 4, "scales", torch.float32, on_gpu=False)
            check_gpu(values, "values")
            if scales is not None:
                check_gpu(scales, "scales")
        check(lib().spmm_plan_set_values(self._h, _ptr(values), _ptr(scales), _stream(stream)))

    def _operands(self, X, Y, n, ldx, ldy):
        n = _ncols(X) if n is None else int(n)
        check_dense(X, self.k, n, self.x, "X", on_gpu=False)
        check_dense(Y, self.m, n, self.y, "Y", on_gpu=False)
        ldx, ldy = _ld(X, ldx, "X"), _ld(Y, ldy, "Y")
        check_gpu(X, "X")
        check_gpu(Y, "Y")
        return n, ldx, ldy

    def run(self, X, Y, n=None, ldx=None, ldy=None, stream=None):
        n, ldx, ldy = self._operands(X, Y, n, ldx, ldy)
        check(lib().spmm_run_static(self._h, n, _ptr(X), ldx, _ptr(Y), ldy, _stream(stream)))
        return Y

    def autotune(self, X, Y, n=None, ldx=None, ldy=None, stream=None):
        """spmm_autotune_static_all: returns (chosen variant, {variant: mean ms})
        over every candidate (a variant is tile width + 256 * kernel form)."""
        n, ldx, ldy = self._operands(X, Y, n, ldx, ldy)
        cap = 8
        vs = (ctypes.c_int32 * cap)()
        ts = (ctypes.c_float * cap)()
        count, best = ctypes.c_int32(), ctypes.c_int32()
        check(lib().spmm_autotune_static_all(self._h, int(n), _ptr(X), int(ldx), _ptr(Y), int(ldy), _stream(stream),
                                             cap, vs, ts, ctypes.byref(count), ctypes.byref(best)))
        return best.value, {int(vs[i]): float(ts[i]) for i in range(count.value)}

    def autotune_widths(self, X, Y, n=None, ldx=None, ldy=None, stream=None):
        """spmm_autotune_static: (chosen variant, {tile width: best mean ms over kernel forms})."""
        n, ldx, ldy = self._operands(X, Y, n, ldx, ldy)
        v = ctypes.c_int32()
        t = (ctypes.c_float * 3)()
        check(lib().spmm_autotune_static(self._h, int(n), _ptr(X), int(ldx), _ptr(Y), int(ldy), _stream(stream),
                                         ctypes.byref(v), t))
        return v.value, {var: float(ms) for var, ms in zip((2, 4, 8), t) if ms >= 0}

    def variant_for(self, n):
        """spmm_plan_variant: the variant a run with n columns uses now (0 = untuned)."""
        v = ctypes.c_int32()
        check(lib().spmm_plan_variant(self._h, int(n), ctypes.byref(v)))
        return v.value

    def export(self):
        inf = self.info()
        row_ptr = np.zeros(self.mb + 1, np.int32)
        col_idx = np.zeros(max(inf["nnzb"], 1), np.int32)
        panel_ptr = np.zeros(inf["num_panels"] + 1, np.int32)
        order = np.zeros(max(inf["nnzb"], 1), np.int32)
        check(lib().spmm_plan_export(self._h, row_ptr.ctypes.data_as(_vp), col_idx.ctypes.data_as(_vp),
                                     panel_ptr.ctypes.data_as(_vp), order.ctypes.data_as(_vp)))
        return {"row_ptr": row_ptr, "col_idx": col_idx[: inf["nnzb"]], "panel_ptr": panel_ptr,
                "order": order[: inf["nnzb"]]}

    @classmethod
    def from_ell(cls, m, k, b, ell_cols, w="f16", x=None, y=None, group_rows=0, num_panels=0, n_hint=0, variant=0):
        """spmm_plan_ell: a plan from a blocked-ELL pattern (int32 [ceil(m/b), width], -1 = empty slot)."""
        x = x or ("f16" if w == "fp8" else w)
        y = y or x
        cols = np.ascontiguousarray(np.asarray(ell_cols, dtype=np.int32))
        mb = -(-int(m) // int(b))
        if cols.ndim != 2 or cols.shape[0] != mb:
            raise ValueError("ell_cols must have shape (ceil(m/b), width)")
        t = cls.__new__(cls)
        t.m, t.k, t.b = int(m), int(k), int(b)
        t.w, t.x, t.y = DTYPE_CODES[w], DTYPE_CODES[x], DTYPE_CODES[y]
        h = _vp()
        opts = _opts(group_rows, num_panels, n_hint, variant)
        check(lib().spmm_plan_ell(t.m, t.k, t.b, int(cols.shape[1]), cols.ctypes.data_as(_vp), t.w, t.x, t.y,
                                  ctypes.byref(opts), ctypes.byref(h)))
        t._h = h
        t.mb, t.kb = mb, -(-t.k // t.b)
        t.ell_width = int(cols.shape[1])
        return t

    def set_values_ell(self, values, scales=None, stream=None):
        """spmm_plan_set_values_ell: values in ELL slot order [ceil(m/b), width, b, b]."""
        import torch
        slots = self.mb * self.ell_width
        if slots:
            check_flat(values, slots * self.b * self.b, _ELEM_BYTES[self.w], "values")
            if scales is not None:
                check_flat(scales, slots, 4, "scales", torch.float32)
        check(lib().spmm_plan_set_values_ell(self._h, _ptr(values), _ptr(scales), _stream(stream)))

    def transpose(self, group_rows=0, num_panels=0, n_hint=0, variant=0):
        """spmm_plan_transpose: the plan of W^T (k x m) with the values transposed."""
        h = _vp()
        opts = _opts(group_rows, num_panels, n_hint, variant)
        check(lib().spmm_plan_transpose(self._h, ctypes.byref(opts), ctypes.byref(h)))
        t = StaticPlan.__new__(StaticPlan)
        t._h = h
        t.m, t.k, t.b = self.k, self.m, self.b
        t.w, t.x, t.y = self.w, self.x, self.y
        t.mb, t.kb = self.kb, self.mb
        t._nnzb_cache = None
        return t

    def sddmm(self, dY, X, G, n=None, stream=None):
        """spmm_sddmm: G[e] = dY[rows of r] X[rows of c]^T on the plan's blocks (FP32 [nnzb, b, b])."""
        import torch
        n = _ncols(X) if n is None else int(n)
        check_dense(dY, self.m, n, self.y, "dY", on_gpu=False)
        check_dense(X, self.k, n, self.x, "X", on_gpu=False)
        check_flat(G, self._nnzb() * self.b * self.b, 4, "G", torch.float32, on_gpu=False)
        for t, name in ((dY, "dY"), (X, "X"), (G, "G")):
            check_gpu(t, name)
        check(lib().spmm_sddmm(self._h, n, _ptr(dY), int(dY.stride(0)), _ptr(X), int(X.stride(0)), _ptr(G),
                               _stream(stream)))
        return G

    def close(self):
        if getattr(self, "_h", None):
            lib().spmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DynamicHandle:
    """spmm_dynamic_create / spmm_run_dynamic."""

    def __init__(self, m, k, b, max_nnzb, w="f16", x=None, y=None, group_rows=0, num_panels=0, n_hint=0):
        x = x or ("f16" if w == "fp8" else w)
        y = y or x
        self.m, self.k, self.b, self.max_nnzb = int(m), int(k), int(b), int(max_nnzb)
        self.w, self.x, self.y = DTYPE_CODES[w], DTYPE_CODES[x], DTYPE_CODES[y]
        self.mb, self.kb = -(-self.m // self.b), -(-self.k // self.b)
        h = _vp()
        opts = _opts(group_rows, num_panels, n_hint)
        check(lib().spmm_dynamic_create(self.m, self.k, self.b, self.max_nnzb, self.w, self.x, self.y,
                                        ctypes.byref(opts), ctypes.byref(h)))
        self._h = h

    def run(self, nnz_dev, rows, cols, values, X, Y, status_dev, scales=None, n=None, ldx=None, ldy=None,
            stream=None):
        torch = _torch()
        n = _ncols(X) if n is None else int(n)
        check_dense(X, self.k, n, self.x, "X", on_gpu=False)
        check_dense(Y, self.m, n, self.y, "Y", on_gpu=False)
        ldx, ldy = _ld(X, ldx, "X"), _ld(Y, ldy, "Y")
        # the index and value buffers are read only up to the device-side count,
        # which the host cannot see; their dtypes and devices are checked
        flat = [(nnz_dev, 1, 4, "nnz_dev", torch.int32), (status_dev, 1, 4, "status_dev", torch.int32),
                (rows, 0, 4, "rows", torch.int32), (cols, 0, 4, "cols", torch.int32),
                (values, 0, _ELEM_BYTES[self.w], "values", None)]
        if scales is not None:
            flat.append((scales, 0, 4, "scales", torch.float32))
        for t, cnt, eb, name, dt in flat:
            check_flat(t, cnt, eb, name, dt, on_gpu=False)
        for t, name in [(X, "X"), (Y, "Y")] + [(f[0], f[3]) for f in flat]:
            check_gpu(t, name)
        check(lib().spmm_run_dynamic(self._h, _ptr(nnz_dev), _ptr(rows), _ptr(cols), _ptr(values), _ptr(scales),
                                     n, _ptr(X), ldx, _ptr(Y), ldy, _ptr(status_dev), _stream(stream)))
        return Y

    def info(self):
        gr, ng, npn = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().spmm_dynamic_info(self._h, ctypes.byref(gr), ctypes.byref(ng), ctypes.byref(npn)))
        return {"group_rows": gr.value, "num_groups": ng.value, "num_panels": npn.value}

    def export(self):
        inf = self.info()
        row_ptr = np.zeros(self.mb + 1, np.int32)
        col_idx = np.zeros(max(self.max_nnzb, 1), np.int32)
        src = np.zeros(max(self.max_nnzb, 1), np.int32)
        panel_ptr = np.zeros(inf["num_panels"] + 1, np.int32)
        nnz = ctypes.c_int64()
        check(lib().spmm_dynamic_export(self._h, row_ptr.ctypes.data_as(_vp), col_idx.ctypes.data_as(_vp),
                                        src.ctypes.data_as(_vp), panel_ptr.ctypes.data_as(_vp), ctypes.byref(nnz)))
        z = nnz.value
        return {"row_ptr": row_ptr, "col_idx": col_idx[:z], "src": src[:z], "panel_ptr": panel_ptr, "nnzb": z}

    def close(self):
        if getattr(self, "_h", None):
            lib().spmm_dynamic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """spmm_group_create / spmm_group_run: many static products in one launch."""

    def __init__(self, max_problems):
        h = _vp()
        check(lib().spmm_group_create(int(max_problems), ctypes.byref(h)))
        self._h = h
        self.max_problems = int(max_problems)

    def run(self, plans, Xs, Ys, ns=None, relu=None, stream=None):
        cnt = len(plans)
        if len(Xs) != cnt or len(Ys) != cnt or (ns is not None and len(ns) != cnt):
            raise ValueError("plans, Xs, Ys and ns must have one entry per problem")
        for i, (p, X, Y) in enumerate(zip(plans, Xs, Ys)):
            n = _ncols(X) if ns is None else int(ns[i])
            check_dense(X, p.k, n, p.x, "X[%d]" % i, on_gpu=False)
            check_dense(Y, p.m, n, p.y, "Y[%d]" % i, on_gpu=False)
        for i, (X, Y) in enumerate(zip(Xs, Ys)):
            check_gpu(X, "X[%d]" % i)
            check_gpu(Y, "Y[%d]" % i)
        P = (_vp * cnt)(*[p._h.value for p in plans])
        N = (ctypes.c_int64 * cnt)(*[(X.shape[1] if ns is None else ns[i]) for i, X in enumerate(Xs)])
        XP = (_vp * cnt)(*[_ptr(X) for X in Xs])
        YP = (_vp * cnt)(*[_ptr(Y) for Y in Ys])
        LX = (ctypes.c_int64 * cnt)(*[X.stride(0) for X in Xs])
        LY = (ctypes.c_int64 * cnt)(*[Y.stride(0) for Y in Ys])
        R = (ctypes.c_uint8 * cnt)(*[1 if (relu and relu[i]) else 0 for i in range(cnt)]) if relu is not None else None
        check(lib().spmm_group_run(self._h, cnt, P, N, XP, LX, YP, LY, R, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().spmm_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """spmm_serve_*: a request loop over a chain of resident sparse layers.

    plans: StaticPlan per layer (None entries allowed when simulate=True);
    dims: feature sizes [num_layers + 1]; relu: per-layer flags."""

    def __init__(self, plans, dims, relu=None, mem_budget_bytes=1 << 30, max_active=64, mode=SERVE_CONTINUOUS,
                 manual=False, simulate=False, max_tokens=0):
        L = len(dims) - 1
        self._plans = plans  # keep the plans alive as long as the server
        P = (_vp * L)(*[(p._h.value if p is not None else None) for p in plans]) if plans is not None else None
        D = (ctypes.c_int64 * (L + 1))(*[int(d) for d in dims])
        R = (ctypes.c_uint8 * L)(*[1 if (relu and relu[i]) else 0 for i in range(L)]) if relu is not None else None
        opts = ServeOpts(int(mem_budget_bytes), int(max_active), int(mode), int(bool(manual)), int(bool(simulate)),
                         int(max_tokens))
        h = _vp()
        check(lib().spmm_serve_create(P, L, D, R, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._keep = {}  # request id -> host buffers kept alive until done
        self.dims = [int(d) for d in dims]
        live = [p for p in (plans or []) if p is not None]
        self._x_bytes = _ELEM_BYTES[live[0].x] if live else None
        self._y_bytes = _ELEM_BYTES[live[-1].y] if live else None

    def submit(self, req_id, n, x_host=None, y_host=None):
        """x_host / y_host: C-contiguous [dims[0], ld] and [dims[-1], ld] host arrays
        (numpy arrays, or torch CPU tensors, pinned for asynchronous copies) with
        ld >= n; None when simulating."""
        def ptr_ld(a, rows, elem, name):
            if a is None:
                return None, int(n)
            if hasattr(a, "data_ptr"):
                if a.is_cuda:
                    raise ValueError("%s must be host memory" % name)
                shape, itemsize = tuple(a.shape), a.element_size()
                strides = tuple(st * itemsize for st in a.stride())
                ptr = a.data_ptr()
            else:
                shape, itemsize, strides, ptr = a.shape, a.itemsize, a.strides, a.ctypes.data
            if len(shape) != 2:
                raise ValueError("%s must be 2-D" % name)
            if elem is not None and itemsize != elem:
                raise ValueError("%s has %d-byte elements, the layer needs %d" % (name, itemsize, elem))
            if shape[1] > 1 and strides[1] != itemsize:
                raise ValueError("%s must have contiguous rows" % name)
            if shape[0] < rows:
                raise ValueError("%s has %d rows, the model needs %d" % (name, shape[0], rows))
            if int(n) > shape[1]:
                raise ValueError("n = %d does not fit the %d columns of %s" % (int(n), shape[1], name))
            return ptr, int(strides[0] // itemsize)
        xp, ldx = ptr_ld(x_host, self.dims[0], self._x_bytes, "x_host")
        yp, ldy = ptr_ld(y_host, self.dims[-1], self._y_bytes, "y_host")
        if ldx != ldy:
            raise ValueError("x_host and y_host must share one leading dimension")
        check(lib().spmm_serve_submit(self._h, int(req_id), int(n), xp, yp, ldx))
        self._keep[int(req_id)] = (x_host, y_host)

    def poll(self, max_items=4096):
        buf = (ServeDone * max_items)()
        k = ctypes.c_int32()
        check(lib().spmm_serve_poll(self._h, buf, int(max_items), ctypes.byref(k)))
        out = []
        for i in range(k.value):
            d = buf[i]
            self._keep.pop(int(d.id), None)
            out.append({"id": int(d.id), "n": int(d.n), "submit_s": d.submit_s, "admit_s": d.admit_s,
                        "done_s": d.done_s})
        return out

    def step(self):
        k = ctypes.c_int32()
        check(lib().spmm_serve_step(self._h, ctypes.byref(k)))
        return k.value

    def drain(self):
        check(lib().spmm_serve_drain(self._h))

    def stats(self):
        st = ServeStats()
        check(lib().spmm_serve_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServeStats._fields_ if f != "reserved"}

    def close(self):
        if getattr(self, "_h", None):
            lib().spmm_serve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_dynamic_noalloc(m, k, b, max_nnzb, nnz_dev, rows, cols, values, X, Y, status_dev, w="f16", x=None, y=None,
                        scales=None, n=None, stream=None):
    """spmm_run_dynamic_noalloc: a dynamic call without a handle; the library
    allocates nothing (its scratch is a fixed device array)."""
    import torch
    x = x or ("f16" if w == "fp8" else w)
    y = y or x
    wc, xc, yc = DTYPE_CODES[w], DTYPE_CODES[x], DTYPE_CODES[y]
    n = _ncols(X) if n is None else int(n)
    check_dense(X, int(k), n, xc, "X", on_gpu=False)
    check_dense(Y, int(m), n, yc, "Y", on_gpu=False)
    flat = [(nnz_dev, 1, 4, "nnz_dev", torch.int32), (status_dev, 1, 4, "status_dev", torch.int32),
            (rows, 0, 4, "rows", torch.int32), (cols, 0, 4, "cols", torch.int32),
            (values, 0, _ELEM_BYTES[wc], "values", None)]
    if scales is not None:
        flat.append((scales, 0, 4, "scales", torch.float32))
    for t, cnt, eb, name, dt in flat:
        check_flat(t, cnt, eb, name, dt, on_gpu=False)
    for t, name in [(X, "X"), (Y, "Y")] + [(f[0], f[3]) for f in flat]:
        check_gpu(t, name)
    check(lib().spmm_run_dynamic_noalloc(int(m), int(k), int(b), int(max_nnzb), wc, xc, yc, _ptr(nnz_dev), _ptr(rows),
                                         _ptr(cols), _ptr(values), _ptr(scales), n, _ptr(X), int(X.stride(0)),
                                         _ptr(Y), int(Y.stride(0)), _ptr(status_dev), _stream(stream)))
    return Y


def clock():
    return lib().spmm_serve_clock()


def speedup_model(m, density, b):
    """spmm_speedup_model: predicted static sparse / dense FP16 speedup on MI355X."""
    out = ctypes.c_double()
    check(lib().spmm_speedup_model(int(m), float(density), int(b), ctypes.byref(out)))
    return out.value
