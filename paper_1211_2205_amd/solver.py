"""Python front end of the MI355X staggered-grid P_N solver.

Thin layer over the C ABI (include/starmap.h): it marshals arguments, wraps
numpy field functions as vectorised callbacks, and lets PyTorch own the
device workspace and the stream.  All computation runs in libstarmap.so.
"""
from __future__ import annotations

import ctypes
import math
from typing import Callable, Optional

import numpy as np

from . import _binding as B

_PREC = {"fp64": B.FP64, "fp32": B.FP32, "bf16": B.BF16}
_BC = {"periodic": B.BC_PERIODIC, "extrapolation": B.BC_EXTRAPOLATION}


def variant_count() -> int:
    """Number of compiled tile variants of the sweep kernel."""
    return int(B.lib().starmap_variant_count())


def num_moments(N: int) -> int:
    return B.check(B.lib().starmap_num_moments(N))


def moment_info(N: int, k: int):
    """(kind 'R'/'I', l, m, gx, gy) of moment k."""
    v = [ctypes.c_int32() for _ in range(5)]
    B.check(B.lib().starmap_moment_info(N, k, *[ctypes.byref(x) for x in v]))
    return ("I" if v[0].value else "R", v[1].value, v[2].value, v[3].value, v[4].value)


def closure_pn(N: int):
    """Dense real M_x, M_y assembled from the library's sparse rows."""
    n = num_moments(N)
    out = []
    for axis in (0, 1):
        cols = np.zeros(4 * n, dtype=np.int32)
        vals = np.zeros(4 * n, dtype=np.float64)
        B.check(B.lib().starmap_closure_pn(N, axis, cols.ctypes.data_as(B._i32p), vals.ctypes.data_as(B._dp)))
        M = np.zeros((n, n))
        for k in range(n):
            for t in range(4):
                if cols[4 * k + t] >= 0:
                    M[k, cols[4 * k + t]] = vals[4 * k + t]
        out.append(M)
    return out[0], out[1]


def spectral_radius(N: int) -> float:
    r = ctypes.c_double()
    B.check(B.lib().starmap_spectral_radius(N, ctypes.byref(r)))
    return r.value


def direction_moments(N: int, omega) -> np.ndarray:
    """Moments of a unit beam delta(Omega - omega) (real basis at omega)."""
    out = np.zeros(num_moments(N))
    ox, oy, oz = (float(v) for v in omega)
    B.check(B.lib().starmap_direction_moments(N, ox, oy, oz, out.ctypes.data_as(B._dp)))
    return out


def _time_callback(a: Callable, keep: list):
    """Wrap a(t) -> float as a C callback; an exception becomes NaN, which the
    library reports as a non-finite time factor."""
    def cb(ctx, t):
        try:
            return float(a(t))
        except Exception:
            import traceback
            traceback.print_exc()
            return math.nan
    c = B.TIME_FN(cb)
    keep.append(c)
    return c


_TERM_FIELD = {"absorption": B.FIELD_ABSORPTION, "scattering": B.FIELD_SCATTERING,
               "scattering_order": B.FIELD_SCATTERING_ORDER, "source": B.FIELD_SOURCE}


def _field_callback(f: Callable, keep: list):
    """Wrap f(t, x, y) -> array as a vectorised C callback."""
    def cb(ctx, t, n, xp, yp, outp):
        try:
            x = np.ctypeslib.as_array(xp, shape=(n,))
            y = np.ctypeslib.as_array(yp, shape=(n,))
            o = np.ctypeslib.as_array(outp, shape=(n,))
            o[:] = np.broadcast_to(np.asarray(f(t, x, y), dtype=np.float64), (n,))
            return 0
        except Exception:  # reported to the library as a callback failure
            import traceback
            traceback.print_exc()
            return 1
    c = B.FIELD_FN(cb)
    keep.append(c)
    return c


class Solver:
    """One P_N problem on one GPU.

    Parameters mirror the paper's problem statement: N, cells n = (nx, ny),
    domain ax = (x0, x1, y0, y1), boundary types, cfl, t_final, precision.
    Device memory is a torch uint8 tensor bound to the library; work runs on
    torch's current stream of the chosen device.
    """

    def __init__(self, N, n, ax, bc=("extrapolation", "extrapolation"), cfl=0.5, t_final=1.0,
                 precision="fp64", device=None, closure="pn"):
        L = B.lib()
        p = B.Problem()
        for i in range(4):
            p.ax[i] = float(ax[i])
        p.n[0], p.n[1] = int(n[0]), int(n[1])
        p.bc[0], p.bc[1] = _BC[bc[0]], _BC[bc[1]]
        p.N = int(N)
        p.cfl = float(cfl)
        p.t_final = float(t_final)
        p.precision = _PREC[precision]
        p.closure = B.CLOSURE_LEARNED if closure == "learned" else B.CLOSURE_PN
        h = ctypes.c_void_p()
        B.check(L.starmap_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._keep = []
        self.N = int(N)
        self.nmom = num_moments(self.N)
        self.precision = precision
        self._device = device
        self._workspace = None

    @classmethod
    def from_problem(cls, prob, device=None, precision=None, closure="pn"):
        """Build from a problem description object with the attributes
        N, n, ax, bc, cfl, t_final, sigma_a, sigma_s0, sigma_sl, source,
        initial, time_dependent, precision (fields are f(t, x, y))."""
        s = cls(prob.N, prob.n, prob.ax, prob.bc, prob.cfl, prob.t_final,
                precision or prob.precision, device=device, closure=closure)
        sep = getattr(prob, "separable", None) or {}
        # with a separable form, the fields it lists carry all time dependence
        td = int(bool(getattr(prob, "time_dependent", False)) and not sep)

        def put(key, index, setter, f):
            terms = sep.get(key) if index is None else sep.get(key, {}).get(index)
            if terms:
                for a, g in terms:
                    s.add_field_term(key, 0 if index is None else index, g, a)
            else:
                setter(f)

        put("absorption", None, lambda f: s.set_absorption(f, td), prob.sigma_a)
        put("scattering", None, lambda f: s.set_scattering(f, td), prob.sigma_s0)
        if getattr(prob, "sigma_sl", None) is not None:
            for l in range(1, prob.N + 1):
                put("scattering_order", l, lambda f, l_=l: s.set_scattering_order(l_, f, td),
                    (lambda l_: (lambda t, x, y: prob.sigma_sl(l_, t, x, y)))(l))
        for k, f in prob.source.items():
            put("source", k, lambda f, k_=k: s.set_source(k_, f, td), f)
        if getattr(prob, "beam_direction", None) is not None:
            # a beam source q(x) delta(Omega - Omega_0): q(x) times each moment's basis value
            w = direction_moments(prob.N, prob.beam_direction)
            for k in range(len(w)):
                if w[k] != 0.0 and k not in prob.source:
                    s.set_source(k, (lambda c: (lambda t, x, y: c * prob.beam_profile(t, x, y)))(float(w[k])), td)
        for k, f in prob.initial.items():
            s.set_initial(k, f)
        if getattr(prob, "filter_damping", None) is not None:
            s.set_filter_damping(prob.filter_damping)
        if getattr(prob, "diffusion", None) is not None:
            s.set_diffusion(prob.diffusion)
        return s

    # ----------------------------------------------------------- fields
    def set_absorption(self, f, time_dependent=0):
        B.check(B.lib().starmap_set_absorption(self._h, _field_callback(f, self._keep), None, int(time_dependent)))

    def set_scattering(self, f, time_dependent=0):
        B.check(B.lib().starmap_set_scattering(self._h, _field_callback(f, self._keep), None, int(time_dependent)))

    def set_scattering_order(self, l, f, time_dependent=0):
        B.check(B.lib().starmap_set_scattering_order(self._h, int(l), _field_callback(f, self._keep), None,
                                                     int(time_dependent)))

    def set_source(self, k, f, time_dependent=0):
        B.check(B.lib().starmap_set_source(self._h, int(k), _field_callback(f, self._keep), None,
                                           int(time_dependent)))

    def add_field_term(self, which, index, g, a):
        """Add a(t) g(x, y) to a field ("absorption", "scattering",
        "scattering_order" with index = l, "source" with index = k); the
        decay and source planes of such fields are formed on the device."""
        B.check(B.lib().starmap_add_field_term(self._h, _TERM_FIELD[which], int(index),
                                               _field_callback(lambda t, x, y: g(x, y), self._keep), None,
                                               _time_callback(a, self._keep), None))

    def set_filter_damping(self, damping):
        """Filtered P_N: damping[l] (l = 0..N) added to the decay of every
        order-l moment; None removes it."""
        if damping is None:
            B.check(B.lib().starmap_set_filter_damping(self._h, None))
            return
        d = np.ascontiguousarray(damping, dtype=np.float64)
        if d.shape != (self.N + 1,):
            raise ValueError(f"filter damping needs N + 1 = {self.N + 1} values")
        B.check(B.lib().starmap_set_filter_damping(self._h, d.ctypes.data_as(B._dp)))

    def set_fused(self, enable=True):
        """Parity-fused passes (orders up to 7): each step's odd and even
        half-steps in one pass over the state; bitwise equal results."""
        B.check(B.lib().starmap_set_fused(self._h, int(bool(enable))))

    def set_diffusion(self, kappa):
        """Diffusion-corrected P_N: kappa(t, x, y) of the diffusion step on the
        order-N moments (sampled once); None removes it."""
        cb = _field_callback(kappa, self._keep) if kappa is not None else B.FIELD_FN()
        B.check(B.lib().starmap_set_diffusion(self._h, cb, None))

    def set_initial(self, k, f):
        B.check(B.lib().starmap_set_initial(self._h, int(k), _field_callback(f, self._keep), None))

    def set_field_array(self, which, k, vals):
        v = np.ascontiguousarray(vals, dtype=np.float64)
        nx, ny, _, _ = self.moment_shape(k)
        assert v.size == nx * ny
        B.check(B.lib().starmap_set_field_array(self._h, int(which), int(k), v.ctypes.data_as(B._dp)))

    # ------------------------------------------------------------ queries
    def moment_shape(self, k):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        x0, y0 = ctypes.c_double(), ctypes.c_double()
        B.check(B.lib().starmap_moment_shape(self._h, int(k), ctypes.byref(a), ctypes.byref(b),
                                             ctypes.byref(x0), ctypes.byref(y0)))
        return a.value, b.value, x0.value, y0.value

    def time(self):
        t, dt = ctypes.c_double(), ctypes.c_double()
        d, tot = ctypes.c_int64(), ctypes.c_int64()
        B.check(B.lib().starmap_time(self._h, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(d), ctypes.byref(tot)))
        return t.value, dt.value, d.value, tot.value

    @property
    def dt(self):
        return self.time()[1]

    @property
    def nsteps(self):
        return self.time()[3]

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        B.check(B.lib().starmap_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    def sweep_bytes(self, parity):
        b = ctypes.c_double()
        B.check(B.lib().starmap_sweep_bytes(self._h, int(parity), ctypes.byref(b)))
        return b.value

    # ------------------------------------------------------------- device
    def bind_torch(self, device=None):
        """Allocate the workspace as a torch tensor and run on torch's current
        stream of that device."""
        import torch
        dev = torch.device(device or self._device or "cuda")
        nbytes = self.workspace_bytes()
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = ws.data_ptr()
        off = (-ptr) % 256
        stream = torch.cuda.current_stream(dev).cuda_stream
        B.check(B.lib().starmap_bind_device(self._h, ctypes.c_void_p(ptr + off), nbytes, ctypes.c_void_p(stream)))
        self._workspace = ws
        return ws

    def advance(self, nsteps):
        B.check(B.lib().starmap_advance(self._h, int(nsteps)))

    def run(self):
        B.check(B.lib().starmap_run(self._h))

    def load_closure(self, params):
        """Load the closure network (flat FP32 parameter blob, see
        include/starmap.h) into a solver created with closure="learned"."""
        w = np.ascontiguousarray(params, dtype=np.float32).ravel()
        B.check(B.lib().starmap_closure_load(self._h, w.ctypes.data_as(B._fp), w.size))

    def closure_samples(self, points, features, targets):
        """Closure inputs and order-6 flux targets at cells points[r] = (i, j)
        of this (order >= 6) solver's current state, written into the float32
        device tensors features (count x 128) and targets (count x 6)."""
        pts = np.ascontiguousarray(points, dtype=np.int32).reshape(-1, 2)
        n = pts.shape[0]
        assert features.is_cuda and targets.is_cuda and features.is_contiguous() and targets.is_contiguous()
        assert features.dtype == targets.dtype and str(features.dtype) == "torch.float32"
        assert features.numel() >= n * 128 and targets.numel() >= n * 6
        B.check(B.lib().starmap_closure_samples(self._h, pts.ctypes.data_as(B._i32p), n,
                                                ctypes.c_void_p(features.data_ptr()),
                                                ctypes.c_void_p(targets.data_ptr())))

    def closure_features(self, points, features, nu=None):
        """Closure inputs (and the stencil norms nu) at cells points[r] = (i, j)
        of this (order >= 5) solver's current state, into float32 device
        tensors features (count x 128) and nu (count)."""
        pts = np.ascontiguousarray(points, dtype=np.int32).reshape(-1, 2)
        n = pts.shape[0]
        assert features.is_cuda and features.is_contiguous() and str(features.dtype) == "torch.float32"
        assert features.numel() >= n * 128
        if nu is not None:
            assert nu.is_cuda and nu.is_contiguous() and str(nu.dtype) == "torch.float32" and nu.numel() >= n
        B.check(B.lib().starmap_closure_features(self._h, pts.ctypes.data_as(B._i32p), n,
                                                 ctypes.c_void_p(features.data_ptr()),
                                                 ctypes.c_void_p(nu.data_ptr() if nu is not None else 0)))

    def reset(self):
        """Back to the initial condition at t = 0."""
        B.check(B.lib().starmap_reset(self._h))

    def sweep(self, parity, tau, nsweeps=1):
        B.check(B.lib().starmap_sweep(self._h, int(parity), float(tau), int(nsweeps)))

    def synchronize(self):
        B.check(B.lib().starmap_synchronize(self._h))

    def get_moment(self, k):
        nx, ny, _, _ = self.moment_shape(k)
        out = np.empty((ny, nx), dtype=np.float64)
        B.check(B.lib().starmap_get_moment(self._h, int(k), out.ctypes.data_as(B._dp)))
        return out

    def moments(self):
        return [self.get_moment(k) for k in range(self.nmom)]

    def get_state(self):
        b = ctypes.c_size_t()
        B.check(B.lib().starmap_state_bytes(self._h, ctypes.byref(b)))
        buf = np.empty(b.value, dtype=np.uint8)
        t, st = ctypes.c_double(), ctypes.c_int64()
        B.check(B.lib().starmap_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), b.value,
                                          ctypes.byref(t), ctypes.byref(st)))
        return buf, t.value, st.value

    def set_state(self, buf, t, step):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        B.check(B.lib().starmap_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size, float(t), int(step)))

    def diagnostics(self, raise_unstable=True):
        m, l2, mx = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        nf = ctypes.c_int32()
        rc = B.lib().starmap_diagnostics(self._h, ctypes.byref(m), ctypes.byref(l2), ctypes.byref(mx), ctypes.byref(nf))
        if rc != B.EUNSTABLE or raise_unstable:
            B.check(rc)
        return {"mass": m.value, "l2": l2.value, "maxabs": mx.value, "nonfinite": nf.value}

    def set_variant(self, v):
        B.check(B.lib().starmap_set_variant(self._h, int(v)))

    def variant(self):
        v, tx, ty = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        B.check(B.lib().starmap_get_variant(self._h, ctypes.byref(v), ctypes.byref(tx), ctypes.byref(ty)))
        return v.value, tx.value, ty.value

    def autotune(self, sweeps=3):
        B.check(B.lib().starmap_autotune(self._h, int(sweeps)))

    def set_closure_fused(self, enable):
        """Closure solvers: network and odd sweep in one kernel (True) or two."""
        B.check(B.lib().starmap_closure_set_fused(self._h, 1 if enable else 0))

    def set_graphs(self, enable):
        """Replay the repeated sweep pairs of advance() from captured HIP graphs."""
        B.check(B.lib().starmap_set_graphs(self._h, 1 if enable else 0))

    def set_chunk_width(self, width):
        """m-range width of the sweep (4, 6 or 8)."""
        B.check(B.lib().starmap_set_range_width(self._h, int(width)))

    def chunk_width(self):
        w = ctypes.c_int32()
        B.check(B.lib().starmap_get_range_width(self._h, ctypes.byref(w)))
        return w.value

    def profile_begin(self):
        B.check(B.lib().starmap_profile_begin(self._h))

    def profile_end(self):
        """(summed sweep-kernel ms, launches, summed algorithmic bytes)."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        B.check(B.lib().starmap_profile_end(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)))
        return ms.value, n.value, b.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            try:
                self.synchronize()
            except B.StarmapError:
                pass
            B.lib().starmap_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several solvers advanced together: instances grouped by order N, one
    launch per sweep and group over the group's instances still running, the
    whole run in one HIP graph.  The solvers must outlive the batch (it keeps
    references to them)."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s._h.value for s in self.solvers])
        self._h = ctypes.c_void_p()
        B.check(B.lib().starmap_batch_create(arr, len(self.solvers), ctypes.byref(self._h)))

    def run(self, use_graph=True):
        """Advance every solver to t_final; returns the last_run record."""
        B.check(B.lib().starmap_batch_run(self._h, 1 if use_graph else 0))
        return self.last_run()

    def last_run(self):
        ms, up, by, nl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
        B.check(B.lib().starmap_batch_last_run(self._h, ctypes.byref(ms), ctypes.byref(up), ctypes.byref(by),
                                               ctypes.byref(nl)))
        return {"ms": ms.value, "updates": up.value, "bytes": by.value, "launches": nl.value}

    def reset(self):
        for s in self.solvers:
            s.reset()

    def set_variant(self, variant, width):
        B.check(B.lib().starmap_batch_set_variant(self._h, int(variant), int(width)))

    def variant(self):
        v, w = ctypes.c_int32(), ctypes.c_int32()
        B.check(B.lib().starmap_batch_get_variant(self._h, ctypes.byref(v), ctypes.byref(w)))
        return v.value, w.value

    def autotune(self, sweeps=3):
        B.check(B.lib().starmap_batch_autotune(self._h, int(sweeps)))

    def groups(self):
        """Per group (ascending N): {"N", "count", "variant", "width"}."""
        n = B.lib().starmap_batch_group_count(self._h)
        B.check(min(n, 0))
        out = []
        for g in range(n):
            N, c, v, w = (ctypes.c_int32() for _ in range(4))
            B.check(B.lib().starmap_batch_get_group(self._h, g, ctypes.byref(N), ctypes.byref(c), ctypes.byref(v),
                                                    ctypes.byref(w)))
            out.append({"N": N.value, "count": c.value, "variant": v.value, "width": w.value})
        return out

    def set_merged(self, merged):
        """One launch per sweep over every group (shared tile variant) or not."""
        B.check(B.lib().starmap_batch_set_merged(self._h, 1 if merged else 0))

    def merged(self):
        return bool(B.check(B.lib().starmap_batch_get_merged(self._h)))

    def set_group_variant(self, group, variant, width):
        B.check(B.lib().starmap_batch_set_group_variant(self._h, int(group), int(variant), int(width)))

    def tile_of(self, i):
        """(variant, width) of the group that solver i belongs to."""
        N = self.solvers[i].N
        g = next(g for g in self.groups() if g["N"] == N)
        return g["variant"], g["width"]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            B.lib().starmap_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The closure network's trainer on the device (forward, backward and Adam
    in the library's kernels).  Batches are float32 torch device tensors;
    work runs on torch's current stream."""

    def __init__(self, max_batch, device=None):
        import torch
        dev = torch.device(device or "cuda")
        self._stream = torch.cuda.current_stream(dev)
        self._h = ctypes.c_void_p()
        B.check(B.lib().starmap_mlp_create(int(max_batch), ctypes.c_void_p(self._stream.cuda_stream),
                                           ctypes.byref(self._h)))
        self.max_batch = int(max_batch)

    @staticmethod
    def _dev(t, cols):
        assert t.is_cuda and t.is_contiguous() and str(t.dtype) == "torch.float32" and t.shape[-1] == cols
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, params):
        w = np.ascontiguousarray(params, dtype=np.float32).ravel()
        B.check(B.lib().starmap_mlp_set_params(self._h, w.ctypes.data_as(B._fp), w.size))

    def params(self):
        w = np.empty(B.CLOSURE_PARAMS, dtype=np.float32)
        B.check(B.lib().starmap_mlp_get_params(self._h, w.ctypes.data_as(B._fp), w.size))
        return w

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=x.device)
        B.check(B.lib().starmap_mlp_forward(self._h, self._dev(x, 128), x.shape[0], self._dev(y, 6)))
        return y

    def gradients(self, x, t):
        g = np.empty(B.CLOSURE_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        B.check(B.lib().starmap_mlp_gradients(self._h, self._dev(x, 128), self._dev(t, 6), x.shape[0],
                                              g.ctypes.data_as(B._fp), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, lr, want_loss=False):
        loss = ctypes.c_double()
        B.check(B.lib().starmap_mlp_train_step(self._h, self._dev(x, 128), self._dev(t, 6), x.shape[0], float(lr),
                                               ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def adam_step(self, grad, lr):
        g = np.ascontiguousarray(grad, dtype=np.float32).ravel()
        B.check(B.lib().starmap_mlp_adam_step(self._h, g.ctypes.data_as(B._fp), float(lr)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            B.lib().starmap_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
