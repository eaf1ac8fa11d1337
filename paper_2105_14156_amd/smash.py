"""ctypes binding of libsmash (include/smash.h): argument marshalling only.

Every step of the multiply runs in the HIP library; this module turns torch
device tensors into the C ABI's pointers and sizes.  Importing it fails
loudly when ``libsmash.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmash.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950) first")

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
STATUS = {0: "SMASH_OK", 1: "SMASH_ERR_INVALID_ARG", 2: "SMASH_ERR_INVALID_CSR", 3: "SMASH_ERR_INDEX_OVERFLOW",
          4: "SMASH_ERR_CAPACITY", 5: "SMASH_ERR_OUT_OF_MEMORY", 6: "SMASH_ERR_HIP", 7: "SMASH_ERR_NO_PLAN"}
F32, F64 = 0, 1
OPT_VALIDATE, OPT_LDS_ROW_MAX, OPT_HEAVY_MODE, OPT_TIMING, OPT_FUSED_SIZING, OPT_GLOBAL_POOL, OPT_ROW_HASH = range(7)
CAPACITY = 4


class CsrDesc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("rows", "products", "nnz_c", "rows_empty", "rows_lds",
                                               "rows_heavy", "heavy_segments", "heavy_dense_chunks",
                                               "global_slots", "nnz_heavy", "nnz_dense", "fused_rows",
                                               "fused_overflow", "fused_capacity", "global_waves",
                                               "global_pool", "fused_entries", "workspace_bytes")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
MLP_FEATURES, MLP_PARAMS = 6, 4673


class TrainArgs(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]

_c = ctypes.c_void_p
_lib.smash_create.argtypes = [ctypes.POINTER(_c), ctypes.c_int]
_lib.smash_destroy.argtypes = [_c]
_lib.smash_destroy.restype = None
_lib.smash_last_error.argtypes = [_c]
_lib.smash_last_error.restype = ctypes.c_char_p
_lib.smash_status_string.argtypes = [ctypes.c_int]
_lib.smash_status_string.restype = ctypes.c_char_p
_lib.smash_set_option.argtypes = [_c, ctypes.c_int, ctypes.c_int64]
_lib.smash_get_option.argtypes = [_c, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
_lib.smash_workspace_size.argtypes = [_c, ctypes.c_int, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc),
                                      ctypes.POINTER(ctypes.c_size_t), _c]
_lib.smash_spgemm_symbolic.argtypes = [_c, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc), _c,
                                       ctypes.POINTER(ctypes.c_int64), _c, ctypes.c_size_t, _c]
_lib.smash_spgemm_numeric.argtypes = [_c, ctypes.c_int, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc), _c, _c, _c,
                                      _c, ctypes.c_size_t, _c]
_lib.smash_spgemm.argtypes = [_c, ctypes.c_int, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc), ALLOC_FN, _c, _c,
                              ctypes.POINTER(_c), ctypes.POINTER(_c), ctypes.POINTER(ctypes.c_int64), _c,
                              ctypes.c_size_t, _c]
_lib.smash_sync.argtypes = [_c, _c]
_lib.smash_spgemm_noalloc.argtypes = [_c, ctypes.c_int, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc), _c, _c, _c,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _c]
NOALLOC_SCRATCH_BYTES = 64 << 20
_lib.smash_get_stats.argtypes = [_c, ctypes.POINTER(Stats)]
_lib.smash_kernel_count.argtypes = []
_lib.smash_kernel_time.argtypes = [_c, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_double)]
_lib.smash_kernel_time_reset.argtypes = [_c]
_lib.smash_features.argtypes = [_c, ctypes.POINTER(CsrDesc), ctypes.POINTER(CsrDesc), _c, _c]
_lib.smash_mlp_predict.argtypes = [_c, ctypes.c_int64, _c, _c, _c, _c, _c]
_lib.smash_mlp_loss_grad.argtypes = [_c, _c, _c, _c, ctypes.c_int64, _c, _c, _c, ctypes.POINTER(ctypes.c_double), _c]
_lib.smash_mlp_train.argtypes = [_c, _c, _c, ctypes.c_int64, _c, _c, _c, ctypes.POINTER(TrainArgs),
                                 ctypes.POINTER(ctypes.c_double), _c]
_lib.smash_predictor_set.argtypes = [_c, _c, _c, ctypes.c_float]
_lib.smash_predictor_load.argtypes = [_c, ctypes.c_char_p]
_lib.smash_spgemm_fused.argtypes = _lib.smash_spgemm.argtypes
_lib.smash_spgemm_fused.restype = ctypes.c_int
for _f in ("smash_features", "smash_mlp_predict", "smash_mlp_loss_grad", "smash_mlp_train", "smash_predictor_set",
           "smash_predictor_load"):
    getattr(_lib, _f).restype = ctypes.c_int
for _f in ("smash_create", "smash_set_option", "smash_get_option", "smash_spgemm_symbolic", "smash_spgemm_numeric",
           "smash_spgemm", "smash_get_stats", "smash_kernel_count", "smash_kernel_time", "smash_kernel_time_reset",
           "smash_workspace_size", "smash_sync", "smash_spgemm_noalloc"):
    getattr(_lib, _f).restype = ctypes.c_int


class BatchConfig(ctypes.Structure):
    _fields_ = [("lds_row_max", ctypes.c_int32), ("table_shift", ctypes.c_int32), ("wide_groups", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("row_hash", ctypes.c_int32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib.smash_batch_plan_create.argtypes = [_c, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(CsrDesc),
                                         ctypes.POINTER(CsrDesc), ctypes.POINTER(BatchConfig), ALLOC_FN, _c,
                                         ctypes.POINTER(_c), _c]
_lib.smash_batch_plan_configure.argtypes = [_c, ctypes.POINTER(BatchConfig), _c]
_lib.smash_batch_plan_get_config.argtypes = [_c, ctypes.POINTER(BatchConfig)]
_lib.smash_batch_plan_outputs.argtypes = [_c, ctypes.POINTER(_c), ctypes.POINTER(_c), ctypes.POINTER(_c),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))]
_lib.smash_batch_plan_run.argtypes = [_c, _c]
_lib.smash_batch_plan_capture.argtypes = [_c, _c]
_lib.smash_batch_plan_launch.argtypes = [_c, _c]
_lib.smash_batch_plan_result.argtypes = [_c, _c, ctypes.POINTER(ctypes.c_int64), _c]
_lib.smash_batch_plan_destroy.argtypes = [_c]
_lib.smash_batch_plan_destroy.restype = None
_lib.smash_batch_autotune.argtypes = [_c, _c, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(BatchConfig),
                                      ctypes.POINTER(ctypes.c_double)]
for _f in ("smash_batch_plan_create", "smash_batch_plan_configure", "smash_batch_plan_get_config",
           "smash_batch_plan_outputs", "smash_batch_plan_run", "smash_batch_plan_capture", "smash_batch_plan_launch",
           "smash_batch_plan_result", "smash_batch_autotune"):
    getattr(_lib, _f).restype = ctypes.c_int


class SmashError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


@dataclasses.dataclass
class DeviceCSR:
    """CSR in device memory (torch tensors: int32 row_ptr/col_idx)."""
    rows: int
    cols: int
    row_ptr: "object"
    col_idx: "object"
    val: "object"

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def desc(self) -> CsrDesc:
        return CsrDesc(self.rows, self.cols, self.nnz, self.row_ptr.data_ptr(),
                       self.col_idx.data_ptr() if self.nnz else 0,
                       self.val.data_ptr() if (self.val is not None and self.nnz) else 0)


def to_device(M, device="cuda", dtype=None) -> DeviceCSR:
    """Copies a host CSR (synthetic.CSR) to the device."""
    import torch
    val = M.val if dtype is None else M.val.astype(dtype)
    return DeviceCSR(M.rows, M.cols,
                     torch.from_numpy(np.ascontiguousarray(M.row_ptr, np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(M.col_idx, np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(val)).to(device))


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported value dtype {t.dtype}")


class Context:
    """One libsmash context on one HIP device."""

    def __init__(self, device: int = 0):
        h = _c()
        st = _lib.smash_create(ctypes.byref(h), int(device))
        if st != OK:
            raise SmashError(st, f"smash_create(device={device}) failed")
        self._h = h
        self.device = int(device)
        self._keep = []
        self._ws = None            # workspace tensor grown on demand (uint8, device)
        self._plan_ws = None       # the workspace of the last symbolic call

    def close(self):
        if getattr(self, "_h", None):
            _lib.smash_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != OK:
            raise SmashError(st, _lib.smash_last_error(self._h).decode())

    def set_option(self, opt: int, value: int):
        self._check(_lib.smash_set_option(self._h, int(opt), int(value)))

    def get_option(self, opt: int) -> int:
        v = ctypes.c_int64()
        self._check(_lib.smash_get_option(self._h, int(opt), ctypes.byref(v)))
        return int(v.value)

    # ------------------------------------------------------------ workspace
    def workspace_size(self, A: DeviceCSR, B: DeviceCSR, stream=None) -> int:
        """Bytes of workspace C = A * B needs (smash_workspace_size)."""
        n = ctypes.c_size_t()
        da, db = A.desc(), B.desc()
        dt = _dtype_code(A.val) if A.val is not None else F32
        self._check(_lib.smash_workspace_size(self._h, dt, ctypes.byref(da), ctypes.byref(db), ctypes.byref(n),
                                              _stream_ptr(stream)))
        return int(n.value)

    def workspace(self, nbytes: int, device="cuda"):
        """A torch uint8 device tensor of at least nbytes (the context's own,
        grown on demand; a grown workspace replaces the old one)."""
        import torch
        nbytes = max(int(nbytes), 256)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self._ws

    @staticmethod
    def _ws_args(ws):
        return (ws.data_ptr(), ws.numel()) if ws is not None and ws.numel() else (None, 0)

    def _with_workspace(self, call, ws, device):
        """Runs call(ws_ptr, ws_bytes); with ws None it uses the context's
        workspace, grown to the size the library reports after CAPACITY."""
        if ws is not None:
            self._check(call(*self._ws_args(ws)))
            return ws
        cur = self._ws
        for _ in range(3):
            st = call(*self._ws_args(cur))
            need = self.stats()["workspace_bytes"] if st == CAPACITY else 0
            if st == CAPACITY and need > (cur.numel() if cur is not None else 0):
                cur = self.workspace(need, device)
                continue
            self._check(st)
            return cur
        self._check(st)
        return cur

    def symbolic(self, A: DeviceCSR, B: DeviceCSR, C_row_ptr, stream=None, ws=None) -> int:
        nnz = ctypes.c_int64()
        da, db = A.desc(), B.desc()
        self._plan_ws = self._with_workspace(
            lambda wp, wb: _lib.smash_spgemm_symbolic(self._h, ctypes.byref(da), ctypes.byref(db),
                                                      C_row_ptr.data_ptr(), ctypes.byref(nnz), wp, wb,
                                                      _stream_ptr(stream)), ws, A.row_ptr.device)
        return int(nnz.value)

    def numeric(self, A: DeviceCSR, B: DeviceCSR, C_row_ptr, C_col, C_val, stream=None, ws=None, check=True):
        """Numeric phase; with check (default) it then synchronises and
        reports what the kernels found (smash_sync)."""
        da, db = A.desc(), B.desc()
        wp, wb = self._ws_args(ws if ws is not None else self._plan_ws)
        self._check(_lib.smash_spgemm_numeric(self._h, _dtype_code(A.val), ctypes.byref(da), ctypes.byref(db),
                                              C_row_ptr.data_ptr(), C_col.data_ptr() if C_col.numel() else 0,
                                              C_val.data_ptr() if C_val.numel() else 0, wp, wb,
                                              _stream_ptr(stream)))
        if check:
            self.sync(stream)

    def spgemm_noalloc(self, A: DeviceCSR, B: DeviceCSR, C_row_ptr, C_col, C_val, stream=None) -> int:
        """smash_spgemm_noalloc into caller buffers (capacity C_col.numel());
        returns nnz(C).  On CAPACITY the raised SmashError carries .nnz."""
        nnz = ctypes.c_int64(-1)
        da, db = A.desc(), B.desc()
        st = _lib.smash_spgemm_noalloc(self._h, _dtype_code(A.val), ctypes.byref(da), ctypes.byref(db),
                                       C_row_ptr.data_ptr(), C_col.data_ptr() if C_col.numel() else 0,
                                       C_val.data_ptr() if C_val.numel() else 0, min(C_col.numel(), C_val.numel()),
                                       ctypes.byref(nnz), _stream_ptr(stream))
        if st != OK:
            err = SmashError(st, _lib.smash_last_error(self._h).decode())
            err.nnz = int(nnz.value)
            raise err
        return int(nnz.value)

    def sync(self, stream=None):
        """smash_sync: waits for the stream, raises what numeric calls found."""
        self._check(_lib.smash_sync(self._h, _stream_ptr(stream)))

    def spgemm_fused(self, A: DeviceCSR, B: DeviceCSR, stream=None, C_row_ptr=None, ws=None) -> DeviceCSR:
        """C = A * B through smash_spgemm_fused (needs an installed predictor)."""
        return self.spgemm(A, B, stream, C_row_ptr, ws=ws, _fn=_lib.smash_spgemm_fused)

    def spgemm(self, A: DeviceCSR, B: DeviceCSR, stream=None, C_row_ptr=None, ws=None, _fn=None) -> DeviceCSR:
        """C = A * B through smash_spgemm; C's arrays and (with ws None) the
        workspace come from torch."""
        import torch
        dev = A.row_ptr.device
        if C_row_ptr is None:
            C_row_ptr = torch.empty(A.rows + 1, dtype=torch.int64, device=dev)
        held = []

        def _alloc(nbytes, _user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
            held.append(t)
            return t.data_ptr()

        cb = ALLOC_FN(_alloc)
        col_p, val_p, nnz = _c(), _c(), ctypes.c_int64()
        da, db = A.desc(), B.desc()
        fn = _fn or _lib.smash_spgemm

        def call(wp, wb):
            held.clear()
            return fn(self._h, _dtype_code(A.val), ctypes.byref(da), ctypes.byref(db), cb, None,
                      C_row_ptr.data_ptr(), ctypes.byref(col_p), ctypes.byref(val_p), ctypes.byref(nnz), wp, wb,
                      _stream_ptr(stream))

        self._plan_ws = self._with_workspace(call, ws, dev)
        n = int(nnz.value)
        # the output buffers are the last two allocations (a fused call first
        # allocates its staging area)
        col = held[-2].view(torch.int32)[:n]
        val = held[-1].view(A.val.dtype)[:n]
        self._keep = held[:-2]      # staging buffers stay alive until the next call
        return DeviceCSR(A.rows, B.cols, C_row_ptr, col, val)

    # ------------------------------------------------------------ predictor
    def features(self, A: DeviceCSR, B: DeviceCSR, stream=None):
        import torch
        out = torch.empty((A.rows, MLP_FEATURES), dtype=torch.float32, device=A.row_ptr.device)
        da, db = A.desc(), B.desc()
        self._check(_lib.smash_features(self._h, ctypes.byref(da), ctypes.byref(db), out.data_ptr() if A.rows else 0,
                                        _stream_ptr(stream)))
        return out

    def mlp_predict(self, feats, params, mean_std, stream=None):
        import torch
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        self._check(_lib.smash_mlp_predict(self._h, feats.shape[0], feats.data_ptr(), params.data_ptr(),
                                           mean_std.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
        return out

    def mlp_loss_grad(self, feats, targets, idx, mean_std, params, stream=None):
        import torch
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device)
        loss = ctypes.c_double()
        self._check(_lib.smash_mlp_loss_grad(self._h, feats.data_ptr(), targets.data_ptr(), idx.data_ptr(),
                                             idx.numel(), mean_std.data_ptr(), params.data_ptr(), grad.data_ptr(),
                                             ctypes.byref(loss), _stream_ptr(stream)))
        return float(loss.value), grad

    def mlp_train(self, feats, targets, mean_std, params, orders, batch, lr=1e-3, beta1=0.9, beta2=0.999,
                  eps=1e-8, stream=None):
        """Trains params (device float32, updated in place); orders: device
        int32 (epochs x n).  Returns the mean batch loss of every epoch."""
        epochs = orders.shape[0]
        args = TrainArgs(epochs, batch, lr, beta1, beta2, eps)
        losses = (ctypes.c_double * epochs)()
        self._check(_lib.smash_mlp_train(self._h, feats.data_ptr(), targets.data_ptr(), targets.numel(),
                                         mean_std.data_ptr(), params.data_ptr(), orders.data_ptr(),
                                         ctypes.byref(args), losses, _stream_ptr(stream)))
        return np.array(list(losses))

    def predictor_set(self, params, mean_std, delta: float):
        p = np.ascontiguousarray(params, np.float32)
        ms = np.ascontiguousarray(mean_std, np.float32)
        self._check(_lib.smash_predictor_set(self._h, p.ctypes.data, ms.ctypes.data, float(delta)))

    def predictor_load(self, path: str = None):
        """Installs a predictor file (default: the weights shipped with the package)."""
        path = path or os.path.join(HERE, "data", "predictor_v2.bin")
        self._check(_lib.smash_predictor_load(self._h, os.fsencode(path)))

    def stats(self) -> dict:
        s = Stats()
        self._check(_lib.smash_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def kernel_times(self) -> dict:
        """{kernel name: (launches, total ms)} with OPT_TIMING on."""
        out = {}
        for i in range(_lib.smash_kernel_count()):
            name, n, ms = ctypes.c_char_p(), ctypes.c_int64(), ctypes.c_double()
            self._check(_lib.smash_kernel_time(self._h, i, ctypes.byref(name), ctypes.byref(n), ctypes.byref(ms)))
            out[name.value.decode()] = (int(n.value), float(ms.value))
        return out

    def reset_kernel_times(self):
        self._check(_lib.smash_kernel_time_reset(self._h))


class BatchPlan:
    """A batch of products C_p = A_p * B_p run as one pipeline
    (smash_batch_plan_*).  The output pool (row pointers over all problems'
    rows, column and value pools) is allocated by torch at creation and held
    here; ``problem(p)`` returns C_p as tensor views of it."""

    def __init__(self, ctx: "Context", As, Bs, config: dict = None, stream=None):
        import torch
        assert len(As) == len(Bs)
        self.ctx = ctx
        self.count = len(As)
        self._inputs = (list(As), list(Bs))         # keep the operands alive
        dt = As[0].val.dtype if As else torch.float32
        self.dtype = dt
        self.dev = As[0].row_ptr.device if As else torch.device("cuda")
        da = (CsrDesc * max(1, self.count))(*[a.desc() for a in As])
        db = (CsrDesc * max(1, self.count))(*[b.desc() for b in Bs])
        self._held = []

        def _alloc(nbytes, _user):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.dev)
            self._held.append(t)
            return t.data_ptr()

        self._cb = ALLOC_FN(_alloc)
        cfg = ctypes.byref(BatchConfig(**config)) if config else None
        h = _c()
        ctx._check(_lib.smash_batch_plan_create(ctx._h, F32 if dt == torch.float32 else F64, self.count, da, db, cfg,
                                                self._cb, None, ctypes.byref(h), _stream_ptr(stream)))
        self._h = h
        cap, rows = ctypes.c_int64(), ctypes.c_int64()
        r0 = ctypes.POINTER(ctypes.c_int64)()
        ctx._check(_lib.smash_batch_plan_outputs(self._h, None, None, None, ctypes.byref(cap), ctypes.byref(rows),
                                                 ctypes.byref(r0)))
        self.capacity, self.total_rows = int(cap.value), int(rows.value)
        self.row0 = np.array([r0[i] for i in range(self.count + 1)], dtype=np.int64)
        crp, ccol, cval = _c(), _c(), _c()
        ctx._check(_lib.smash_batch_plan_outputs(self._h, ctypes.byref(crp), ctypes.byref(ccol), ctypes.byref(cval),
                                                 None, None, None))
        by_ptr = {t.data_ptr(): t for t in self._held}
        self.C_row_ptr = by_ptr[crp.value].view(torch.int64)[:self.total_rows + 1]
        self.C_col = by_ptr[ccol.value].view(torch.int32)[:self.capacity]
        self.C_val = by_ptr[cval.value].view(dt)[:self.capacity]

    def close(self):
        if getattr(self, "_h", None):
            _lib.smash_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def configure(self, config: dict, stream=None):
        self.ctx._check(_lib.smash_batch_plan_configure(self._h, ctypes.byref(BatchConfig(**config)),
                                                        _stream_ptr(stream)))

    def config(self) -> dict:
        g = BatchConfig()
        self.ctx._check(_lib.smash_batch_plan_get_config(self._h, ctypes.byref(g)))
        return g.as_dict()

    def run(self, stream=None):
        self.ctx._check(_lib.smash_batch_plan_run(self._h, _stream_ptr(stream)))

    def capture(self, stream):
        self.ctx._check(_lib.smash_batch_plan_capture(self._h, _stream_ptr(stream)))

    def launch(self, stream=None):
        self.ctx._check(_lib.smash_batch_plan_launch(self._h, _stream_ptr(stream)))

    def result(self, stream=None):
        """(total entries, per-problem entries); synchronises the stream."""
        tot = ctypes.c_int64()
        per = np.zeros(max(1, self.count), dtype=np.int64)
        self.ctx._check(_lib.smash_batch_plan_result(self._h, _stream_ptr(stream), ctypes.byref(tot),
                                                     per.ctypes.data))
        return int(tot.value), per[:self.count]

    def autotune(self, reps=3, cache_path=None, stream=None):
        """Returns (chosen configuration, its mean ms or 0 on a cache hit)."""
        g, ms = BatchConfig(), ctypes.c_double()
        self.ctx._check(_lib.smash_batch_autotune(self._h, _stream_ptr(stream), reps,
                                                  os.fsencode(cache_path) if cache_path else None,
                                                  ctypes.byref(g), ctypes.byref(ms)))
        return g.as_dict(), float(ms.value)

    def problem(self, p: int) -> DeviceCSR:
        """C_p as views of the pool (row pointers rebased to its first entry)."""
        r0, r1 = int(self.row0[p]), int(self.row0[p + 1])
        rp = self.C_row_ptr[r0:r1 + 1]
        base = int(rp[0].item())
        n = int(rp[-1].item()) - base
        return DeviceCSR(r1 - r0, int(self._inputs[1][p].cols), rp - base, self.C_col[base:base + n],
                         self.C_val[base:base + n])


def status_string(code: int) -> str:
    return _lib.smash_status_string(int(code)).decode()


def exported_symbols():
    """Names of the C entry points this binding expects."""
    return [n for n in dir(_lib) if n.startswith("smash_")]
