"""Python binding of libfks: the fast spectral Boltzmann collision operator Q(f, f)
and the exact-shift transport of the Fast Kinetic Scheme on MI355X (gfx950).

Every step of the computation runs in the HIP kernels behind the C ABI
(include/fks.h).  This module only marshals arguments: torch tensors provide device
memory and the current stream.  There is no CPU fallback; if libfks.so is missing,
every call raises.
"""

import ctypes
import threading

import torch

from . import _lib
from ._lib import (FKS_ALLOW_OVERLAP, FKS_CONSERVE, FKS_F32, FKS_F64, FKS_HARD_SPHERES, FKS_VHS,  # noqa: F401
                   FKSError)

__all__ = ["Plan", "Transport", "step", "step_ex", "collide_grouped", "FKSError", "library_path", "profile_start",
           "profile_stop", "Graph", "Surrogate"]

_DT = {"f32": (FKS_F32, torch.float32), "f64": (FKS_F64, torch.float64)}


def library_path():
    return _lib.LIB_PATH


def _stream_ptr(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


# Stream capture (Graph): while a graph records on this thread, the wrappers allocate
# nothing (an allocation inside the recording would be freed when the wrapper returns
# while the graph keeps writing to it) and every plan, transport and tensor they are given
# is held by the graph until it is destroyed.
_capture = threading.local()


def _recording():
    return getattr(_capture, "graph", None)


def _hold(*objs):
    g = _recording()
    if g is not None:
        g._keep.extend(o for o in objs if o is not None)


def _new_like(t, name):
    if _recording() is not None:
        raise FKSError(-1, f"inside a Graph recording, pass {name} explicitly (no allocation while recording)")
    return torch.empty_like(t)


def _no_recording(what):
    if _recording() is not None:
        raise FKSError(-1, f"{what} synchronises the host and cannot be recorded in a Graph")


class Plan:
    """A collision-operator plan: FP64 host tables built by the library, device tables
    and workspace allocated here (torch) and bound once."""

    def __init__(self, n, L, R, kernel="hard_spheres", alpha=0.0, C=0.25, a1=4, a2=4, n_radial=8,
                 dtype="f32", conserve=False, allow_overlap=False, max_cells=1024, device="cuda",
                 stream=None):
        L_ = _lib.lib()
        self.n, self.L, self.R = int(n), float(L), float(R)
        self.dtype_code, self.torch_dtype = _DT[dtype]
        self.device = torch.device(device)
        flags = (FKS_CONSERVE if conserve else 0) | (FKS_ALLOW_OVERLAP if allow_overlap else 0)
        desc = _lib.CollideDesc(n=self.n, kernel=FKS_HARD_SPHERES if kernel == "hard_spheres" else FKS_VHS,
                                L=self.L, R=self.R, alpha=float(alpha), C=float(C), a1=int(a1), a2=int(a2),
                                n_radial=int(n_radial), dtype=self.dtype_code, flags=flags, reserved=0)
        h = ctypes.c_void_p()
        _lib.check(L_.fks_plan_create(ctypes.byref(desc), int(max_cells), ctypes.byref(h)))
        self._h = h
        self.max_cells = int(max_cells)
        tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(L_.fks_plan_sizes(h, ctypes.byref(tb), ctypes.byref(wb)))
        nt, pad = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(L_.fks_plan_info(h, ctypes.byref(nt), ctypes.byref(pad)))
        self.n_terms, self.pad = nt.value, pad.value
        self.table_bytes, self.workspace_bytes = tb.value, wb.value
        self.tables = torch.empty(max(tb.value, 1), dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(max(wb.value, 1), dtype=torch.uint8, device=self.device)
        _lib.check(L_.fks_plan_bind(h, _ptr(self.tables), tb.value, _ptr(self.workspace), wb.value,
                                    _stream_ptr(stream)))

    @property
    def handle(self):
        return self._h

    def _check_f(self, f, name="f"):
        if not (f.is_cuda and f.dtype == self.torch_dtype and f.is_contiguous()):
            raise FKSError(-1, f"{name} must be a contiguous {self.torch_dtype} device tensor")
        if f.dim() < 3 or tuple(f.shape[-3:]) != (self.n,) * 3:
            raise FKSError(-1, f"{name} must have shape [..., {self.n}, {self.n}, {self.n}]")
        return f.numel() // self.n ** 3

    def collide(self, f, q=None, stream=None):
        cells = self._check_f(f)
        if q is None:
            q = _new_like(f, "q")
        self._check_f(q, "q")
        _hold(self, f, q)
        _lib.check(_lib.lib().fks_collide(self._h, _ptr(f), _ptr(q), cells, _stream_ptr(stream)))
        return q

    def relax(self, f_in, dt, f_out=None, q=None, moments=None, stream=None):
        cells = self._check_f(f_in, "f_in")
        if f_out is None:
            f_out = _new_like(f_in, "f_out")
        self._check_f(f_out, "f_out")
        if q is not None:
            self._check_f(q, "q")
        _hold(self, f_in, f_out, q, moments)
        if moments is not None and not (moments.is_cuda and moments.dtype == torch.float64
                                        and moments.numel() >= 5 * cells):
            raise FKSError(-1, "moments must be a float64 device tensor with 5 entries per cell")
        _lib.check(_lib.lib().fks_relax(self._h, _ptr(f_in), _ptr(f_out), _ptr(q), float(dt), cells,
                                        _ptr(moments), _stream_ptr(stream)))
        return f_out

    def schedule(self):
        sl, xc = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.lib().fks_plan_schedule(self._h, ctypes.byref(sl), ctypes.byref(xc)))
        return sl.value, xc.value

    def set_schedule(self, slabs, xcd_map=1):
        _lib.check(_lib.lib().fks_plan_set_schedule(self._h, int(slabs), int(xcd_map)))

    def term_groups(self):
        """(groups in effect, maximum for this plan)."""
        tg, mx = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.lib().fks_plan_get_term_groups(self._h, ctypes.byref(tg), ctypes.byref(mx)))
        return tg.value, mx.value

    def set_term_groups(self, tg):
        _lib.check(_lib.lib().fks_plan_set_term_groups(self._h, int(tg)))

    def autotune(self, f, q=None, cache_path=None, stream=None):
        """Time the compiled slab schedules on f and keep the fastest (optional cache file)."""
        _no_recording("autotune")
        cells = self._check_f(f)
        if q is None:
            q = torch.empty_like(f)
        path = cache_path.encode() if cache_path else None
        _lib.check(_lib.lib().fks_plan_autotune(self._h, _ptr(f), _ptr(q), cells, path, _stream_ptr(stream)))
        return self.schedule()

    def heun(self, f, dt, n_steps=1, tmp=None, stream=None):
        """n_steps Heun steps of df/dt = Q(f) in place on f (device scratch tmp: 2 buffers)."""
        cells = self._check_f(f)
        if tmp is None:
            tmp = (_new_like(f, "tmp"), _new_like(f, "tmp"))
        _hold(self, f, *tmp)
        _lib.check(_lib.lib().fks_heun(self._h, _ptr(f), _ptr(tmp[0]), _ptr(tmp[1]), float(dt), int(n_steps),
                                       cells, _stream_ptr(stream)))
        return f

    def moments(self, f, out=None, stream=None):
        cells = self._check_f(f)
        if out is None:
            if _recording() is not None:
                raise FKSError(-1, "inside a Graph recording, pass out explicitly")
            out = torch.empty((cells, 5), dtype=torch.float64, device=f.device)
        _hold(self, f, out)
        _lib.check(_lib.lib().fks_moments(self._h, _ptr(f), cells, _ptr(out), _stream_ptr(stream)))
        return out

    def noneq(self, f, out=None, stream=None):
        """Normalised non-equilibrium residual per cell (deviatoric stress and heat flux), FP64."""
        cells = self._check_f(f)
        if out is None:
            if _recording() is not None:
                raise FKSError(-1, "inside a Graph recording, pass out explicitly")
            out = torch.empty((cells,), dtype=torch.float64, device=f.device)
        _hold(self, f, out)
        _lib.check(_lib.lib().fks_noneq(self._h, _ptr(f), cells, _ptr(out), _stream_ptr(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib._lib.fks_plan_destroy(h)
            self._h = None


class Surrogate:
    """Fourier-mode MLP surrogate of Q with spectral fallback (fks_sur_* in include/fks.h).

    Parameters, Adam state and activations live in two device buffers allocated here and
    bound once; every computation runs in the library's kernels."""

    def __init__(self, n, modes=8, width=1024, max_batch=1024, out_scale=1.0, center=False, device="cuda",
                 stream=None):
        L_ = _lib.lib()
        h = ctypes.c_void_p()
        flags = _lib.FKS_SUR_CENTER if center else 0
        _lib.check(L_.fks_sur_create(int(n), int(modes), int(width), int(max_batch), float(out_scale), flags,
                                     ctypes.byref(h)))
        self.out_scale = float(out_scale)
        self.center = bool(center)
        self._h = h
        self.n, self.modes, self.width, self.max_batch = int(n), int(modes), int(width), int(max_batch)
        self.n_in, self.n_out = 2 * self.modes ** 3, self.n ** 3
        self.device = torch.device(device)
        pb, wb, npar = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
        _lib.check(L_.fks_sur_sizes(h, ctypes.byref(pb), ctypes.byref(wb), ctypes.byref(npar)))
        self.n_params = npar.value
        self.params_buf = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        _lib.check(L_.fks_sur_bind(h, _ptr(self.params_buf), pb.value, _ptr(self.workspace), wb.value,
                                   _stream_ptr(stream)))
        self._loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def shapes(self):
        w, i, o = self.width, self.n_in, self.n_out
        return [(w, i), (w,), (w, w), (w,), (o, w), (o,)]

    def set_params(self, params, stream=None):
        """params: W1, b1, W2, b2, W3, b3 (array-likes, weights [out][in]); resets Adam."""
        flat = torch.cat([torch.as_tensor(p, dtype=torch.float32).reshape(-1) for p in params]).contiguous()
        if flat.numel() != self.n_params:
            raise FKSError(-1, f"expected {self.n_params} parameters, got {flat.numel()}")
        _lib.check(_lib.lib().fks_sur_set_params(self._h, ctypes.c_void_p(flat.data_ptr()), _stream_ptr(stream)))

    def _get(self, which, stream=None):
        flat = torch.empty(self.n_params, dtype=torch.float32)
        _lib.check(_lib.lib().fks_sur_get(self._h, which, ctypes.c_void_p(flat.data_ptr()), _stream_ptr(stream)))
        out, o = [], 0
        for shp in self.shapes():
            k = 1
            for d in shp:
                k *= d
            out.append(flat[o:o + k].reshape(shp).numpy())
            o += k
        return out

    def get_params(self, stream=None):
        return self._get(0, stream)

    def get_grads(self, stream=None):
        return self._get(1, stream)

    def features(self, plan, f, x=None, rho=None, mom=None, stream=None):
        """(x, rho, mom): BF16 features, FP32 densities and FP64 moments of f."""
        cells = plan._check_f(f)
        if _recording() is not None and (x is None or rho is None or mom is None):
            raise FKSError(-1, "inside a Graph recording, pass x, rho and mom explicitly")
        _hold(self, plan, f, x, rho, mom)
        if x is None:
            x = torch.empty((cells, self.n_in), dtype=torch.bfloat16, device=f.device)
        if rho is None:
            rho = torch.empty(cells, dtype=torch.float32, device=f.device)
        if mom is None:
            mom = torch.empty((cells, 5), dtype=torch.float64, device=f.device)
        if not (x.dtype == torch.bfloat16 and x.is_contiguous() and x.numel() >= cells * self.n_in):
            raise FKSError(-1, "x must be a contiguous bfloat16 tensor of [cells, 2 modes^3]")
        if not (mom.dtype == torch.float64 and mom.is_contiguous() and mom.numel() >= 5 * cells):
            raise FKSError(-1, "mom must be a contiguous float64 tensor of [cells, 5]")
        _lib.check(_lib.lib().fks_sur_features(self._h, plan.handle, _ptr(f), _ptr(x), _ptr(rho), _ptr(mom), cells,
                                               _stream_ptr(stream)))
        return x, rho, mom

    def targets(self, plan, q, rho, mom=None, t=None, stream=None):
        cells = q.numel() // self.n_out
        if t is None:
            t = _new_like(q, "t")
        _hold(self, plan, q, rho, mom, t)
        _lib.check(_lib.lib().fks_sur_targets(self._h, plan.handle, _ptr(q), _ptr(rho), _ptr(mom), _ptr(t), cells,
                                              _stream_ptr(stream)))
        return t

    def forward(self, x, y=None, stream=None):
        batch = x.shape[0]
        if y is None:
            if _recording() is not None:
                raise FKSError(-1, "inside a Graph recording, pass y explicitly")
            y = torch.empty((batch, self.n_out), dtype=torch.float32, device=x.device)
        _hold(self, x, y)
        _lib.check(_lib.lib().fks_sur_forward(self._h, _ptr(x), _ptr(y), batch, _stream_ptr(stream)))
        return y

    def train_step(self, x, t, lr, update=True, loss=None, stream=None):
        """One forward/backward (and Adam step if update); returns the device loss tensor."""
        batch = x.shape[0]
        loss = self._loss if loss is None else loss
        _hold(self, x, t, loss)
        _lib.check(_lib.lib().fks_sur_train_step(self._h, _ptr(x), _ptr(t), batch, float(lr), int(bool(update)),
                                                 _ptr(loss), _stream_ptr(stream)))
        return loss

    def infer(self, plan, f, q=None, threshold=1e-3, indicator=None, stream=None):
        """Q of FP32 cells f: surrogate, indicator, spectral fallback where it exceeds
        threshold (threshold < 0: none).  Returns (q, number of fallback cells)."""
        _no_recording("Surrogate.infer")
        cells = plan._check_f(f)
        if q is None:
            q = torch.empty_like(f)
        nf = ctypes.c_int64()
        _lib.check(_lib.lib().fks_sur_infer(self._h, plan.handle, _ptr(f), _ptr(q), cells, float(threshold),
                                            ctypes.byref(nf), _ptr(indicator), _stream_ptr(stream)))
        return q, nf.value

    def infer_ranked(self, plan, f, fallback_frac, q=None, indicator=None, stream=None):
        """Q of FP32 cells f: surrogate, with the spectral fallback for the share fallback_frac
        of each chunk's cells that have the largest absolute residual (relative moment
        residual times ||Q||).  Returns (q, number of fallback cells)."""
        _no_recording("Surrogate.infer_ranked")
        cells = plan._check_f(f)
        if q is None:
            q = torch.empty_like(f)
        nf = ctypes.c_int64()
        _lib.check(_lib.lib().fks_sur_infer_ranked(self._h, plan.handle, _ptr(f), _ptr(q), cells,
                                                   float(fallback_frac), ctypes.byref(nf), _ptr(indicator),
                                                   _stream_ptr(stream)))
        return q, nf.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib._lib.fks_sur_destroy(h)
            self._h = None


class Transport:
    """Exact-shift transport on a periodic box of cells (device offsets state)."""

    def __init__(self, n, L, shape, dx, device="cuda", stream=None):
        L_ = _lib.lib()
        self.n, self.L, self.shape, self.dx = int(n), float(L), tuple(int(s) for s in shape), float(dx)
        h = ctypes.c_void_p()
        _lib.check(L_.fks_xport_create(self.n, self.L, *self.shape, self.dx, ctypes.byref(h)))
        self._h = h
        sb = ctypes.c_size_t()
        _lib.check(L_.fks_xport_sizes(h, ctypes.byref(sb)))
        self.state = torch.empty(sb.value, dtype=torch.uint8, device=device)
        _lib.check(L_.fks_xport_bind(h, _ptr(self.state), sb.value, _stream_ptr(stream)))

    @property
    def handle(self):
        return self._h

    def offsets(self):
        """(s [nv,3] float64, o [nv,3] int32) views of the device state."""
        nv = self.n ** 3
        s_bytes = (nv * 24 + 255) // 256 * 256
        s = self.state[: nv * 24].view(torch.float64).view(nv, 3)
        o = self.state[s_bytes: s_bytes + nv * 12].view(torch.int32).view(nv, 3)
        return s, o

    def __call__(self, f_in, f_out=None, dt=0.0, stream=None):
        if f_out is None:
            f_out = _new_like(f_in, "f_out")
        _hold(self, f_in, f_out)
        code = FKS_F32 if f_in.dtype == torch.float32 else FKS_F64
        _lib.check(_lib.lib().fks_transport(self._h, _ptr(f_in), _ptr(f_out), code, float(dt),
                                            _stream_ptr(stream)))
        return f_out

    def advance(self, dt, stream=None):
        """Advance the offsets by dt without moving f (the shifts stay pending)."""
        _hold(self)
        _lib.check(_lib.lib().fks_transport_ex(self._h, None, None, FKS_F32, float(dt), 0, _stream_ptr(stream)))

    def materialize(self, f_in, f_out=None, stream=None):
        """f_out = f_in moved by the shifts pending since f was last moved."""
        if f_out is None:
            f_out = _new_like(f_in, "f_out")
        _hold(self, f_in, f_out)
        code = FKS_F32 if f_in.dtype == torch.float32 else FKS_F64
        _lib.check(_lib.lib().fks_transport_ex(self._h, _ptr(f_in), _ptr(f_out), code, 0.0, 1,
                                               _stream_ptr(stream)))
        return f_out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib._lib.fks_xport_destroy(h)
            self._h = None


def step(plan, xport, f, dt, n_steps=1, f_tmp=None, moments=None, stream=None):
    """n_steps split steps (transport, then Euler collision) in place on f."""
    if f_tmp is None:
        f_tmp = _new_like(f, "f_tmp")
    _hold(plan, xport, f, f_tmp, moments)
    _lib.check(_lib.lib().fks_step(plan.handle, xport.handle, _ptr(f), _ptr(f_tmp), float(dt), int(n_steps),
                                   _ptr(moments), _stream_ptr(stream)))
    return f


def _check_cells5(t, cells, name):
    if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                              and t.numel() >= 5 * cells):
        raise FKSError(-1, f"{name} must be a contiguous float64 device tensor with 5 entries per cell")


def step_ex(plan, xport, f, dt, n_steps=1, f_tmp=None, collision="boltzmann", integrator="euler", nu=0.0,
            nu_density=False, mu=0.0, cons=None, prim=None, moments=None, q_last=None, stream=None):
    """n_steps FKS steps in place on f with the options of fks_step_ex: collision "boltzmann" or
    "bgk" (frequency nu, times the density if nu_density), integrator "euler" or "exp"
    (penalty mu for Boltzmann), conservative variables cons (in/out, eq. DM_update), primitive
    variables prim, direct moments, and the collision operator of the last step q_last."""
    cells = plan._check_f(f)
    if f_tmp is None:
        f_tmp = _new_like(f, "f_tmp")
    plan._check_f(f_tmp, "f_tmp")
    _hold(plan, xport, f, f_tmp, cons, prim, moments, q_last)
    if q_last is not None:
        plan._check_f(q_last, "q_last")
    for t, name in ((cons, "cons"), (prim, "prim"), (moments, "moments")):
        _check_cells5(t, cells, name)
    o = _lib.StepOpts(collision={"boltzmann": _lib.FKS_COLL_BOLTZMANN, "bgk": _lib.FKS_COLL_BGK}[collision],
                      integrator={"euler": _lib.FKS_INT_EULER, "exp": _lib.FKS_INT_EXP}[integrator],
                      nu=float(nu), nu_density=int(bool(nu_density)), reserved=0, mu=float(mu),
                      d_cons=_ptr(cons), d_prim=_ptr(prim), d_moments=_ptr(moments), q_last=_ptr(q_last))
    _lib.check(_lib.lib().fks_step_ex(plan.handle, xport.handle, _ptr(f), _ptr(f_tmp), float(dt), int(n_steps),
                                      ctypes.byref(o), _stream_ptr(stream)))
    return f


def collide_grouped(plans, fs, qs=None, stream=None):
    """Uneven batch: group g evaluates Q on fs[g] with plans[g] (one call, one stream)."""
    g = len(plans)
    if qs is None:
        qs = [_new_like(f, "qs") for f in fs]
    _hold(*plans, *fs, *qs)
    cells = [p._check_f(f) for p, f in zip(plans, fs)]
    VP = ctypes.c_void_p
    arr_p = (VP * g)(*[p.handle for p in plans])
    arr_f = (VP * g)(*[f.data_ptr() for f in fs])
    arr_q = (VP * g)(*[q.data_ptr() for q in qs])
    arr_n = (ctypes.c_int64 * g)(*cells)
    _lib.check(_lib.lib().fks_collide_grouped(arr_p, g, arr_f, arr_q, arr_n, _stream_ptr(stream)))
    return qs


def profile_start():
    _lib.check(_lib.lib().fks_profile_start())


def profile_stop():
    """{slot name: (total ms, launches)} for the launches since profile_start (host syncs)."""
    st = _lib.ProfileStats()
    _lib.check(_lib.lib().fks_profile_stop(ctypes.byref(st)))
    return {name: (st.total_ms[i], st.launches[i]) for i, name in enumerate(_lib.PROFILE_SLOTS)}


class Graph:
    """Stream capture of library calls into one hipGraph.

        with Graph(stream) as g:      # records, runs nothing
            plan.collide(f, q, stream=stream)
        g.launch()                    # replays on the same stream
    """

    def __init__(self, stream=None):
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self._h = None
        self._keep = []     # plans, transports and tensors the recording uses

    def __enter__(self):
        if _recording() is not None:
            raise FKSError(-1, "a Graph is already recording on this thread")
        _lib.check(_lib.lib().fks_graph_begin(_stream_ptr(self.stream)))
        _capture.graph = self
        return self

    def __exit__(self, exc_type, exc, tb):
        _capture.graph = None
        h = ctypes.c_void_p()
        status = _lib.lib().fks_graph_end(_stream_ptr(self.stream), ctypes.byref(h))
        if exc_type is None:
            _lib.check(status)
            self._h = h
        else:
            if status == 0:
                _lib.lib().fks_graph_destroy(h)
            self._keep = []
        return False

    def launch(self):
        _lib.check(_lib.lib().fks_graph_launch(self._h, _stream_ptr(self.stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib._lib is not None:
            _lib._lib.fks_graph_destroy(h)
            self._h = None
        self._keep = []
