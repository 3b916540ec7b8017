"""Python front end of librte: the same calls as the C ABI, with torch tensors
for device memory and torch streams.  Marshalling only -- every step of the
solve runs in the library's HIP kernels."""
import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import check, lib

_KERNEL = {"auto": L.HG_AUTO, "flatland": L.HG_FLATLAND, "sphere": L.HG_SPHERE}
PRECOND = {"none": L.PC_NONE, "bf16": L.PC_MGNET_BF16, "fp32": L.PC_MGNET_FP32, "bj": L.PC_BLOCK_JACOBI}


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Model:
    """An MGN1 weights blob parsed by mgnet_load."""

    def __init__(self, blob):
        blob = bytes(blob)
        h = C.c_void_p()
        buf = C.create_string_buffer(blob, len(blob))
        check(lib().mgnet_load(buf, len(blob), C.byref(h)))
        self._h = h
        d = (C.c_int * 8)()
        check(lib().mgnet_describe(h, d))
        (self.dim, self.ndir, self.c0, self.levels, self.nu_pre, self.nu_post,
         self.nu_coarse, self.coef_ch) = list(d)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().mgnet_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """rte_build_operator over a problem dict (see rte_inputs.configs)."""

    def __init__(self, prob, model=None, stream=None):
        dirs = _f64(prob["dirs"])
        w = _f64(prob["weights"])
        st, sa, q = _f64(prob["sigma_t"]), _f64(prob["sigma_a"]), _f64(prob["q"])
        eps = prob["eps"]
        eps_arr = None if np.isscalar(eps) else _f64(eps)
        inflow = None if prob.get("inflow") is None else _f64(prob["inflow"])
        g = L.Geometry()
        g.dim = prob["dim"]
        nx, ny, nz = prob["n"]
        g.n[0], g.n[1], g.n[2] = nx, ny, nz
        g.ndir = dirs.shape[0]
        g.dirs = _ptr(dirs)
        g.weights = _ptr(w)
        g.g = float(prob["g"])
        g.kernel = _KERNEL[prob.get("kernel", "auto")]
        g.scheme = {"upwind": L.SCHEME_UPWIND, "tfps": L.SCHEME_TFPS}[prob.get("scheme", "upwind")]
        m = L.Medium()
        m.sigma_t, m.sigma_a, m.q = _ptr(st), _ptr(sa), _ptr(q)
        m.eps = _ptr(eps_arr) if eps_arr is not None else None
        m.eps_scalar = float(eps) if eps_arr is None else 0.0
        m.inflow = _ptr(inflow) if inflow is not None else None
        m.inflow_face_stride = inflow.shape[-1] if inflow is not None else 0
        h = C.c_void_p()
        check(lib().rte_build_operator(C.byref(g), C.byref(m), model.handle if model else None,
                                       _stream(stream) if _cuda_ok() else None, C.byref(h)))
        self._h = h
        self.model = model
        info = L.OperatorInfo()
        check(lib().rte_operator_get_info(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in info._fields_}
        self.n = info.n
        self.cells = info.cells
        self.ndir = info.ndir

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().rte_operator_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inspection
    def array(self, which, level=0, stream=None):
        torch = _torch()
        if which == L.ARR_RHS:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        elif which == L.ARR_SCATTER:
            out = torch.empty(self.ndir * self.ndir, dtype=torch.float64, device="cuda")
        elif which == L.ARR_SIGMA:
            out = torch.empty(2 * self.cells, dtype=torch.float64, device="cuda")
        else:
            C0 = self.model.c0 << level
            cl = self.cells >> (self.info["dim"] * level)
            out = torch.empty(cl * C0, dtype=torch.float32, device="cuda")
        check(lib().rte_operator_copy_array(self._h, which, level, _dptr(out),
                                            out.numel() * out.element_size(), _stream(stream)))
        return out

    def rhs(self, stream=None):
        return self.array(L.ARR_RHS, stream=stream)

    # ---- operator
    def apply(self, x, y=None, stream=None):
        torch = _torch()
        prec = L.FP64 if x.dtype == torch.float64 else L.FP32
        if y is None:
            y = torch.empty_like(x)
        check(lib().rte_apply(self._h, _dptr(x), _dptr(y), prec, _stream(stream)))
        return y

    def cell_values(self, x, psi=None, stream=None):
        """psi at the cell centres, [ndir][cells] FP64 (rte_cell_values)."""
        torch = _torch()
        if psi is None:
            psi = torch.empty(self.ndir * self.cells, dtype=torch.float64, device="cuda")
        check(lib().rte_cell_values(self._h, _dptr(x), _dptr(psi), _stream(stream)))
        return psi

    def residual(self, x, r=None, stream=None):
        torch = _torch()
        if r is None:
            r = torch.empty_like(x)
        check(lib().rte_residual(self._h, _dptr(x), _dptr(r), _stream(stream)))
        return r

    # ---- preconditioner
    def precond_workspace(self, model):
        nb = C.c_size_t()
        check(lib().rte_precond_workspace_bytes(self._h, model.handle, C.byref(nb)))
        return nb.value

    def precond(self, model, v, mode="bf16", z=None, workspace=None, stream=None):
        """z = M(v): the MgNet V-cycle ("bf16", "fp32") or Block-Jacobi ("bj", no model)."""
        torch = _torch()
        if z is None:
            z = torch.empty(self.n, dtype=torch.float32, device="cuda")
        if mode == "bj":
            check(lib().rte_precond_apply(self._h, model.handle if model else None, PRECOND[mode], _dptr(v),
                                          _dptr(z), None, 0, _stream(stream)))
            return z
        if workspace is None:
            workspace = torch.empty(self.precond_workspace(model), dtype=torch.uint8, device="cuda")
        check(lib().rte_precond_apply(self._h, model.handle, PRECOND[mode], _dptr(v), _dptr(z),
                                      _dptr(workspace), workspace.numel(), _stream(stream)))
        return z

    def precond_noalloc(self, model, v, mode="bf16", z=None, stream=None):
        """z = M(v) with the V-cycle activations in the library's own device array
        (rte_precond_apply_noalloc): no workspace, no device allocation in the call."""
        torch = _torch()
        if z is None:
            z = torch.empty(self.n, dtype=torch.float32, device="cuda")
        check(lib().rte_precond_apply_noalloc(self._h, model.handle, PRECOND[mode], _dptr(v), _dptr(z),
                                              _stream(stream)))
        return z

    # ---- solve
    def opts(self, restart=30, rtol=1e-6, max_iters=20000, precond="bf16", x0=None, b=None):
        o = L.SolveOpts()
        o.restart = int(restart)
        o.rtol = float(rtol)
        o.max_iters = int(max_iters)
        o.precond = PRECOND[precond] if isinstance(precond, str) else int(precond)
        o.x0 = x0.data_ptr() if x0 is not None else None
        o.b = b.data_ptr() if b is not None else None
        return o

    def workspace_bytes(self, model=None, **kw):
        o = self.opts(**kw)
        nb = C.c_size_t()
        check(lib().rte_workspace_bytes(self._h, model.handle if model else None, C.byref(o), C.byref(nb)))
        return nb.value

    def solve(self, model=None, psi=None, workspace=None, stream=None, raise_on_noconv=False, **kw):
        """Returns (psi tensor [n] float64, stats dict)."""
        torch = _torch()
        if kw.get("precond", "bf16") in ("bf16", "fp32") and model is None:
            model = self.model
        o = self.opts(**kw)
        if psi is None:
            psi = torch.empty(self.n, dtype=torch.float64, device="cuda")
        if workspace is None:
            nb = C.c_size_t()
            check(lib().rte_workspace_bytes(self._h, model.handle if model else None, C.byref(o),
                                            C.byref(nb)))
            workspace = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        st = L.SolveStats()
        allow = () if raise_on_noconv else (L.RTE_ENOCONV, L.RTE_EBREAKDOWN)
        check(lib().rte_solve(self._h, model.handle if model else None, C.byref(o), _dptr(workspace),
                              workspace.numel(), _dptr(psi), C.byref(st), _stream(stream)), allow)
        return psi, st.as_dict()


class Atfps:
    """The adaptive TFPS maps of a TFPS operator (rte_atfps_build): compressed residual,
    layer reconstruction and filtered loss, evaluated on the device."""

    def __init__(self, op, delta):
        h = C.c_void_p()
        check(lib().rte_atfps_build(op.handle, float(delta), C.byref(h)))
        self._h = h
        self.op = op
        nk, nr, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().rte_atfps_get_info(h, C.byref(nk), C.byref(nr), C.byref(nnz)))
        self.n_kept, self.n_rows, self.nnz = nk.value, nr.value, nnz.value

    def residual(self, alpha, r=None, stream=None):
        """r = b_d - A_d alpha, [n_rows] FP64."""
        torch = _torch()
        if r is None:
            r = torch.empty(self.n_rows, dtype=torch.float64, device="cuda")
        check(lib().rte_atfps_residual(self._h, _dptr(alpha), _dptr(r), _stream(stream)))
        return r

    def reconstruct(self, alpha, coef=None, stream=None):
        """All coefficients [cells][2 ndir] FP64 from the kept ones."""
        torch = _torch()
        if coef is None:
            coef = torch.empty(self.op.n, dtype=torch.float64, device="cuda")
        check(lib().rte_atfps_reconstruct(self._h, _dptr(alpha), _dptr(coef), _stream(stream)))
        return coef

    def filtered_loss(self, psi, rho=None, stream=None):
        """(rho, loss): rho = b_d - A_d D_d psi and its 2-norm (a device scalar)."""
        torch = _torch()
        if rho is None:
            rho = torch.empty(self.n_rows, dtype=torch.float64, device="cuda")
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        check(lib().rte_atfps_filtered_loss(self._h, _dptr(psi), _dptr(rho), _dptr(loss), _stream(stream)))
        return rho, loss

    def close(self):
        if getattr(self, "_h", None):
            lib().rte_atfps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over a caller-owned device arena."""

    def __init__(self, arena_bytes, max_slots=8):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        check(lib().rte_server_create(_dptr(self.arena), self.arena.numel(), int(max_slots), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, op, psi, model=None, **kw):
        o = op.opts(**kw)
        t = C.c_uint64()
        check(lib().rte_submit(self._h, op.handle, model.handle if model else None, C.byref(o),
                               _dptr(psi), C.byref(t)))
        self._keep[t.value] = (op, model, psi, kw.get("x0"), kw.get("b"))
        return t.value

    def submit_many(self, requests):
        """Queue several solves at once (rte_submit_many): `requests` is a list of
        (op, psi, model, kwargs) tuples; returns their tickets in order."""
        n = len(requests)
        if n == 0:
            return []
        ops = (C.c_void_p * n)(*[op.handle for op, _, _, _ in requests])
        models = (C.c_void_p * n)(*[(m.handle if m else None) for _, _, m, _ in requests])
        opts = (L.SolveOpts * n)(*[op.opts(**kw) for op, _, _, kw in requests])
        outs = (C.c_void_p * n)(*[_dptr(psi) for _, psi, _, _ in requests])
        tickets = (C.c_uint64 * n)()
        check(lib().rte_submit_many(self._h, n, ops, models, opts, outs, tickets))
        for (op, psi, m, kw), t in zip(requests, tickets):
            self._keep[t] = (op, m, psi, kw.get("x0"), kw.get("b"))
        return list(tickets)

    def poll(self, ticket):
        """None while running; (status, stats dict) once finished."""
        st = L.SolveStats()
        code = lib().rte_poll(self._h, C.c_uint64(ticket), C.byref(st))
        if code == L.RTE_EAGAIN:
            return None
        if code == L.RTE_ENOTFOUND:
            check(code)
        self._keep.pop(ticket, None)
        return code, st.as_dict()

    def query(self):
        s = L.ServerStats()
        check(lib().rte_server_query(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def close(self):
        if getattr(self, "_h", None):
            check(lib().rte_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prof_enable(cls, every=1):
    """Time every `every`-th launch of a kernel class with HIP events (0 = off)."""
    check(lib().rte_prof_enable(int(cls), int(every)))


def prof_query(cls):
    """(total ms, timed launches, algorithmic work, algorithmic bytes) since the last reset."""
    ms = C.c_double()
    cnt = C.c_int64()
    work = C.c_double()
    nbytes = C.c_double()
    check(lib().rte_prof_query(int(cls), C.byref(ms), C.byref(cnt), C.byref(work), C.byref(nbytes)))
    return ms.value, cnt.value, work.value, nbytes.value


def prof_query_keys(cls):
    """{key: (total ms, timed launches, work, bytes)} for every key with timed launches
    (for convolutions the key is floor(log2(output channels)))."""
    out = {}
    for key in range(16):
        ms = C.c_double()
        cnt = C.c_int64()
        work = C.c_double()
        nbytes = C.c_double()
        check(lib().rte_prof_query_key(int(cls), key, C.byref(ms), C.byref(cnt), C.byref(work), C.byref(nbytes)))
        if cnt.value:
            out[key] = (ms.value, cnt.value, work.value, nbytes.value)
    return out


def prof_reset():
    check(lib().rte_prof_reset())


def _cuda_ok():
    try:
        return _torch().cuda.is_available()
    except Exception:
        return False
