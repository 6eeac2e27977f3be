"""MI355X (gfx950) solver for cone programs by ADMM on the homogeneous
self-dual embedding (O'Donoghue, Chu, Parikh, Boyd).

Thin Python binding over the C ABI of ``libhsd.so`` (include/hsd.h).
PyTorch provides device memory and the stream; every step of the method
runs in the library's HIP kernels.  There is no CPU path: using this module
without the built library or without a GPU raises.
"""

from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from ctypes import byref, c_double, c_int64, c_size_t, c_void_p

import numpy as np

from . import _lib

__all__ = ["Solver", "BatchSolver", "MLP", "project_cone", "default_settings", "STATUS_NAMES"]

STATUS_NAMES = _lib.STATUS_NAMES


def _torch():
    import torch
    return torch


# Handles still open when the interpreter exits are closed by an atexit hook,
# which runs before interpreter finalisation and before the C library's own
# exit handlers (the HIP runtime's teardown, a profiler's finalisation).  A
# handle collected during finalisation itself makes no HIP call: its host
# metadata is left to the process exit.
_LIVE = weakref.WeakSet()


def _close_all() -> None:
    for h in list(_LIVE):
        try:
            h.close()
        except Exception:
            pass


atexit.register(_close_all)


class _Handle:
    """Base of the handle classes: close() is idempotent, the objects are
    context managers, and they are closed at interpreter exit."""

    _h = None

    def _register(self):
        _LIVE.add(self)

    def close(self):
        raise NotImplementedError

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound at definition: module globals may already be gone when a
        # handle is collected late in interpreter shutdown)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def default_settings() -> dict:
    lib = _lib.load()
    st = _lib.HsdSettings()
    lib.hsd_default_settings(byref(st))
    return {name: getattr(st, name) for name, _ in st._fields_}


def _settings(**kw) -> _lib.HsdSettings:
    lib = _lib.load()
    st = _lib.HsdSettings()
    lib.hsd_default_settings(byref(st))
    for k, v in kw.items():
        if not hasattr(st, k):
            raise TypeError(f"unknown setting {k!r}")
        setattr(st, k, v)
    return st


def _csr_to_device(A, device):
    """Accepts a scipy sparse matrix or (indptr, indices, data, (m, n)) and
    returns int32/int32/float64 device tensors plus (m, n)."""
    torch = _torch()
    if isinstance(A, tuple) and isinstance(A[0], torch.Tensor):
        indptr, indices, data, shape = A
        return (indptr.to(device=device, dtype=torch.int32).contiguous(),
                indices.to(device=device, dtype=torch.int32).contiguous(),
                data.to(device=device, dtype=torch.float64).contiguous(),
                int(shape[0]), int(shape[1]))
    if hasattr(A, "tocsr"):
        A = A.tocsr()
        indptr, indices, data, shape = A.indptr, A.indices, A.data, A.shape
    else:
        indptr, indices, data, shape = A
    m, n = int(shape[0]), int(shape[1])
    rp = torch.as_tensor(np.asarray(indptr, dtype=np.int32), device=device)
    ci = torch.as_tensor(np.asarray(indices, dtype=np.int32), device=device)
    va = torch.as_tensor(np.asarray(data, dtype=np.float64), device=device)
    return rp, ci, va, m, n


def _dev_vec(x, device):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device=device).contiguous()


def _aligned_workspace(nbytes: int, device):
    torch = _torch()
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (buf.data_ptr() + 255) // 256 * 256
    return buf, ptr


def _stream_ptr(device):
    torch = _torch()
    return c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver(_Handle):
    """One cone program set up on the GPU.

    ``A`` is a scipy sparse matrix (or (indptr, indices, data, shape)),
    ``b`` and ``c`` are vectors, ``cone`` a dict with keys f, l, q, s, ep, ed
    (row order zero, nonnegative, second-order, PSD scaled svec, exponential,
    dual exponential).  Keyword arguments set fields of hsd_settings_t.
    """

    def __init__(self, A, b, c, cone, device="cuda", **settings):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device(device)
        rp, ci, va, m, n = _csr_to_device(A, self.device)
        self.m, self.n = m, n
        self._b = _dev_vec(b, self.device)
        self._c = _dev_vec(c, self.device)
        self.settings = _settings(**settings)
        self._K, self._keep = _lib.make_cone(cone)
        csr = _lib.HsdCsr(m=m, n=n, nnz=int(ci.numel()), row_ptr=rp.data_ptr(),
                          col_idx=ci.data_ptr(), val=va.data_ptr())
        nbytes = c_size_t(0)
        _lib.check(self.lib.hsd_workspace_bytes(byref(csr), byref(self._K), byref(self.settings),
                                                byref(nbytes)))
        self._ws, ws_ptr = _aligned_workspace(nbytes.value, self.device)
        self.ws_bytes = nbytes.value
        h = c_void_p()
        _lib.check(self.lib.hsd_setup(byref(csr), c_void_p(self._b.data_ptr()),
                                      c_void_p(self._c.data_ptr()), byref(self._K),
                                      byref(self.settings), c_void_p(ws_ptr), nbytes,
                                      _stream_ptr(self.device), byref(h)))
        self._h = h
        self._register()

    def solve(self):
        """Returns (x, y, s, info) with device tensors and an info dict."""
        torch = _torch()
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        y = torch.empty(self.m, dtype=torch.float64, device=self.device)
        s = torch.empty(self.m, dtype=torch.float64, device=self.device)
        info = _lib.HsdInfo()
        _lib.check(self.lib.hsd_solve(self._h, c_void_p(x.data_ptr()), c_void_p(y.data_ptr()),
                                      c_void_p(s.data_ptr()), byref(info)))
        return x, y, s, info.to_dict()

    def warm_start(self, x, y, s):
        xs = [_dev_vec(v, self.device) for v in (x, y, s)]
        _lib.check(self.lib.hsd_warm_start(self._h, *[c_void_p(v.data_ptr()) for v in xs]))
        self._hold = xs

    def start_from_q(self, q):
        qd = _dev_vec(q, self.device)
        _lib.check(self.lib.hsd_start_from_q(self._h, c_void_p(qd.data_ptr())))
        self._hold = qd

    def update_b(self, b):
        """New b for the same A and c (Sect. 4.2 repeated solves)."""
        self._b = _dev_vec(b, self.device)
        _lib.check(self.lib.hsd_update_b(self._h, c_void_p(self._b.data_ptr())))

    def update_bc(self, b, c):
        """New b and c for the same A (Sect. 4.2 repeated solves)."""
        self._b = _dev_vec(b, self.device)
        self._c = _dev_vec(c, self.device)
        _lib.check(self.lib.hsd_update_bc(self._h, c_void_p(self._b.data_ptr()),
                                          c_void_p(self._c.data_ptr())))

    def get_state(self, carry: bool = True) -> dict:
        """State where the last solve or iterate stopped: u, v (n+m+1),
        z_x (n), k, and with ``carry`` the carried products (2m)."""
        torch = _torch()
        N = self.n + self.m + 1
        u = torch.empty(N, dtype=torch.float64, device=self.device)
        v = torch.empty(N, dtype=torch.float64, device=self.device)
        zx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        cr = torch.empty(2 * self.m, dtype=torch.float64, device=self.device) if carry else None
        k = ctypes.c_int32(0)
        _lib.check(self.lib.hsd_get_state(self._h, c_void_p(u.data_ptr()), c_void_p(v.data_ptr()),
                                          c_void_p(zx.data_ptr()),
                                          c_void_p(cr.data_ptr() if cr is not None else None),
                                          byref(k)))
        return {"u": u, "v": v, "zx": zx, "carry": cr, "k": int(k.value)}

    def set_state(self, state: dict, carry: bool = True):
        """Start the next solve or iterate from a state of ``get_state``."""
        u, v, zx = (_dev_vec(state[k], self.device) for k in ("u", "v", "zx"))
        cr = state.get("carry") if carry else None
        cr = _dev_vec(cr, self.device) if cr is not None else None
        _lib.check(self.lib.hsd_set_state(self._h, c_void_p(u.data_ptr()), c_void_p(v.data_ptr()),
                                          c_void_p(zx.data_ptr()),
                                          c_void_p(cr.data_ptr() if cr is not None else None),
                                          int(state["k"])))
        self._hold = (u, v, zx, cr)

    def update_settings(self, **kw):
        st = _lib.HsdSettings()
        ctypes.memmove(ctypes.addressof(st), ctypes.addressof(self.settings), ctypes.sizeof(st))
        for k, v in kw.items():
            if not hasattr(st, k):
                raise TypeError(f"unknown setting {k!r}")
            setattr(st, k, v)
        _lib.check(self.lib.hsd_update_settings(self._h, byref(st)))
        self.settings = st

    def iterate(self, count: int):
        """(U, V): iterates k = 0..count as rows, scaled variables."""
        torch = _torch()
        N = self.n + self.m + 1
        U = torch.empty((count + 1, N), dtype=torch.float64, device=self.device)
        V = torch.empty((count + 1, N), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.hsd_iterate(self._h, int(count), c_void_p(U.data_ptr()),
                                        c_void_p(V.data_ptr())))
        return U, V

    def scaling(self):
        torch = _torch()
        D = torch.empty(self.m, dtype=torch.float64, device=self.device)
        E = torch.empty(self.n, dtype=torch.float64, device=self.device)
        sig, rho = c_double(), c_double()
        _lib.check(self.lib.hsd_get_scaling(self._h, c_void_p(D.data_ptr()), c_void_p(E.data_ptr()),
                                            byref(sig), byref(rho)))
        return D, E, sig.value, rho.value

    def launch(self) -> dict:
        """The launch shape the handle uses (hsd_get_launch)."""
        out = _lib.HsdLaunch()
        _lib.check(self.lib.hsd_get_launch(self._h, byref(out)))
        return out.to_dict()

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hsd_finish(self._h)
            self._h = None



def project_cone(cone, x, dual: bool = False, device="cuda"):
    """Pi_K(x) (or Pi_{K*}(x)) with the library's projection kernels."""
    torch = _torch()
    lib = _lib.load()
    dev = torch.device(device)
    xd = _dev_vec(x, dev)
    out = torch.empty_like(xd)
    K, keep = _lib.make_cone(cone)
    _lib.check(lib.hsd_project_cone(byref(K), int(xd.numel()), c_void_p(xd.data_ptr()),
                                    c_void_p(out.data_ptr()), 1 if dual else 0, _stream_ptr(dev)))
    return out


class BatchSolver(_Handle):
    """Many independent programs solved in one persistent launch (one
    workgroup per program).  ``problems`` is a list of (A, b, c, cone)."""

    def __init__(self, problems, device="cuda", **settings):
        import scipy.sparse as sp
        mats = [sp.csr_matrix(p[0]) for p in problems]
        big = sp.block_diag(mats, format="csr")
        self._setup(big, [M.shape for M in mats], [p[1] for p in problems],
                    [p[2] for p in problems], [p[3] for p in problems], device, settings)

    @classmethod
    def shared(cls, A, bs, c, cone, device="cuda", **settings):
        """B programs with the same A, c and cone and different b (the rows
        of ``bs``).  The block-diagonal matrix is assembled on the device."""
        torch = _torch()
        obj = cls.__new__(cls)
        dev = torch.device(device)
        A = A.tocsr()
        B = int(bs.shape[0])
        m, n = A.shape
        nnz = int(A.nnz)
        rp = torch.as_tensor(np.asarray(A.indptr, dtype=np.int64), device=dev)
        ci = torch.as_tensor(np.asarray(A.indices, dtype=np.int64), device=dev)
        va = torch.as_tensor(np.asarray(A.data, dtype=np.float64), device=dev)
        k = torch.arange(B, device=dev, dtype=torch.int64)
        rp_big = torch.cat([(rp[:-1][None, :] + nnz * k[:, None]).reshape(-1),
                            torch.tensor([B * nnz], device=dev, dtype=torch.int64)])
        ci_big = (ci[None, :] + n * k[:, None]).reshape(-1)
        va_big = va.repeat(B)
        big = (rp_big.to(torch.int32), ci_big.to(torch.int32), va_big, (B * m, B * n))
        bcat = _dev_vec(bs, dev).reshape(-1)
        ccat = _dev_vec(c, dev).repeat(B)
        obj._setup(big, [(m, n)] * B, bcat, ccat, [cone] * B, device, settings)
        return obj

    def _setup_from_block(self, big, problems, device="cuda", **settings):
        """Set up from an already assembled block-diagonal matrix; offsets
        come from the shapes of the problems' A."""
        self._setup(big, [p[0].shape for p in problems], [p[1] for p in problems],
                    [p[2] for p in problems], [p[3] for p in problems], device, settings)

    def _setup(self, big, shapes, bs, cs, cones_in, device, settings):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.B = len(shapes)
        self.row_off = np.zeros(self.B + 1, dtype=np.int64)
        self.col_off = np.zeros(self.B + 1, dtype=np.int64)
        for i, (mi, ni) in enumerate(shapes):
            self.row_off[i + 1] = self.row_off[i] + mi
            self.col_off[i + 1] = self.col_off[i] + ni
        rp, ci, va, m, n = _csr_to_device(big, self.device)
        self.m, self.n = m, n
        if isinstance(bs, list):
            bs = np.concatenate([np.asarray(v, dtype=np.float64) for v in bs])
            cs = np.concatenate([np.asarray(v, dtype=np.float64) for v in cs])
        self._b = _dev_vec(bs, self.device)
        self._c = _dev_vec(cs, self.device)
        self.settings = _settings(**settings)
        cones = [_lib.make_cone(k) for k in cones_in]
        self._keep = [k[1] for k in cones]
        self._K = (_lib.HsdCone * self.B)(*[k[0] for k in cones])
        ro = (c_int64 * (self.B + 1))(*self.row_off.tolist())
        co = (c_int64 * (self.B + 1))(*self.col_off.tolist())
        self._ro, self._co = ro, co
        csr = _lib.HsdCsr(m=m, n=n, nnz=int(ci.numel()), row_ptr=rp.data_ptr(),
                          col_idx=ci.data_ptr(), val=va.data_ptr())
        nbytes = c_size_t(0)
        _lib.check(self.lib.hsd_batch_workspace_bytes(self.B, byref(csr), ro, co, self._K,
                                                      byref(self.settings), byref(nbytes)))
        self._ws, ws_ptr = _aligned_workspace(nbytes.value, self.device)
        h = c_void_p()
        _lib.check(self.lib.hsd_batch_setup(self.B, byref(csr), ro, co, c_void_p(self._b.data_ptr()),
                                            c_void_p(self._c.data_ptr()), self._K,
                                            byref(self.settings), c_void_p(ws_ptr), nbytes,
                                            _stream_ptr(self.device), byref(h)))
        self._h = h
        self._register()

    def solve(self):
        torch = _torch()
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        y = torch.empty(self.m, dtype=torch.float64, device=self.device)
        s = torch.empty(self.m, dtype=torch.float64, device=self.device)
        infos = (_lib.HsdInfo * self.B)()
        _lib.check(self.lib.hsd_batch_solve(self._h, c_void_p(x.data_ptr()), c_void_p(y.data_ptr()),
                                            c_void_p(s.data_ptr()), infos))
        return x, y, s, [i.to_dict() for i in infos]

    def state(self):
        """(u, v) the last solve ended on, in each program's scaled variables
        (device FP64; program i at row_off[i] + col_off[i] + i onwards)."""
        torch = _torch()
        L = int(self.row_off[-1] + self.col_off[-1] + self.B)
        u = torch.empty(L, dtype=torch.float64, device=self.device)
        v = torch.empty(L, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.hsd_batch_get_state(self._h, c_void_p(u.data_ptr()), c_void_p(v.data_ptr())))
        return u, v

    def split(self, vec, kind: str):
        off = self.col_off if kind == "x" else self.row_off
        return [vec[off[i]:off[i + 1]] for i in range(self.B)]

    def launch(self) -> dict:
        """The launch shape of the batched handle (hsd_batch_get_launch)."""
        out = _lib.HsdLaunch()
        _lib.check(self.lib.hsd_batch_get_launch(self._h, byref(out)))
        return out.to_dict()

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hsd_batch_finish(self._h)
            self._h = None



class MLP(_Handle):
    """The warm-start network on the GPU (own FP32 kernels; GEMMs on MFMA).
    Sizes n_in -> n_hidden -> n_hidden -> n_out, batches up to max_batch."""

    def __init__(self, n_in, n_hidden, n_out, max_batch, device="cuda"):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.n_in, self.n_hidden, self.n_out, self.max_batch = n_in, n_hidden, n_out, max_batch
        nb = c_size_t(0)
        _lib.check(self.lib.hsd_mlp_workspace_bytes(n_in, n_hidden, n_out, max_batch, byref(nb)))
        self._ws, ptr = _aligned_workspace(nb.value, self.device)
        h = c_void_p()
        _lib.check(self.lib.hsd_mlp_create(n_in, n_hidden, n_out, max_batch, c_void_p(ptr), nb,
                                           _stream_ptr(self.device), byref(h)))
        self._h = h
        self._register()
        self.P = int(self.lib.hsd_mlp_param_count(h))
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def _f32(self, x):
        torch = _torch()
        if isinstance(x, torch.Tensor):
            return x.to(device=self.device, dtype=torch.float32).contiguous()
        return torch.as_tensor(np.asarray(x, dtype=np.float32), device=self.device).contiguous()

    def set_params(self, p):
        self._p_in = self._f32(p)
        assert self._p_in.numel() == self.P
        _lib.check(self.lib.hsd_mlp_set_params(self._h, c_void_p(self._p_in.data_ptr())))

    def params(self):
        torch = _torch()
        out = torch.empty(self.P, dtype=torch.float32, device=self.device)
        _lib.check(self.lib.hsd_mlp_get_params(self._h, c_void_p(out.data_ptr())))
        return out

    def forward(self, x):
        torch = _torch()
        x = self._f32(x)
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=self.device)
        _lib.check(self.lib.hsd_mlp_forward(self._h, int(x.shape[0]), c_void_p(x.data_ptr()),
                                            c_void_p(y.data_ptr())))
        return y

    def gradients(self, x, t):
        torch = _torch()
        x, t = self._f32(x), self._f32(t)
        g = torch.empty(self.P, dtype=torch.float32, device=self.device)
        _lib.check(self.lib.hsd_mlp_gradients(self._h, int(x.shape[0]), c_void_p(x.data_ptr()),
                                              c_void_p(t.data_ptr()), c_void_p(g.data_ptr()),
                                              c_void_p(self._loss.data_ptr())))
        return g, self._loss.clone()

    def train_step(self, x, t, lr):
        x, t = self._f32(x), self._f32(t)
        _lib.check(self.lib.hsd_mlp_train_step(self._h, int(x.shape[0]), c_void_p(x.data_ptr()),
                                               c_void_p(t.data_ptr()), ctypes.c_float(lr),
                                               c_void_p(self._loss.data_ptr())))
        return self._loss

    def close(self):
        if getattr(self, "_h", None):
            self.lib.hsd_mlp_destroy(self._h)
            self._h = None

