"""Python front end of the library: a ``Plan`` owns the C plan and a torch
workspace on the GPU and forwards every call to the HIP library."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N

try:
    import torch
except ImportError:  # pragma: no cover - torch is required for device memory
    torch = None


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """One problem (``Problem``), solver settings (``Solver``) and precision
    ("fp64" or "fp32": FP32 bulk with FP64 tracing and norms)."""

    def __init__(self, problem, solver, precision="fp64", device="cuda", adjoint=False):
        if torch is None:
            raise N.NativeError("torch is required for device memory")
        self.pr, self.sv, self.precision = problem, solver, precision
        self.adjoint_enabled = bool(adjoint)
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.S = problem.nx if problem.dim == 1 else problem.nx * problem.nx
        desc, self._keep = N.make_desc(problem, solver, precision, adjoint)
        self._desc = desc
        h = C.c_void_p()
        N.check(N.lib().slm_plan_create(C.byref(desc), C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        N.check(N.lib().slm_plan_workspace_size(self.h, C.byref(nb)), self.h)
        self.ws_bytes = nb.value
        nl = C.c_int()
        Ns = (C.c_int * N.MAX_LEVELS)()
        ms = (C.c_int * N.MAX_LEVELS)()
        N.check(N.lib().slm_plan_levels(self.h, C.byref(nl), Ns, ms, N.MAX_LEVELS), self.h)
        self.L = nl.value
        self.N = [Ns[i] for i in range(self.L)]
        self.m = [ms[i] for i in range(self.L)]
        self.ws = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                N.lib().slm_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ------------------------------------------------------------ setup
    def setup(self, stream=None):
        if self.ws is None:
            # over-allocate by 256 bytes and align (the ABI wants 256-byte alignment)
            self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws_raw.data_ptr()) % 256
            self.ws = self._ws_raw[off:off + self.ws_bytes]
        N.check(N.lib().slm_plan_setup(self.h, _ptr(self.ws), self.ws_bytes, _stream(stream)), self.h)
        return self

    def _view(self, ptr, nbytes, dtype, shape):
        off = ptr - self.ws.data_ptr()
        assert 0 <= off and off + nbytes <= self.ws_bytes
        return self.ws[off:off + nbytes].view(dtype).reshape(shape)

    def level_arrays(self, level):
        """(displacement [dim][N][S], sigma [dim][N][S] or None) as views of
        the workspace."""
        dd, ds = C.c_void_p(), C.c_void_p()
        f32 = C.c_int()
        N.check(N.lib().slm_level_arrays(self.h, level, C.byref(dd), C.byref(f32), C.byref(ds)), self.h)
        dim, Nl = self.pr.dim, self.N[level]
        dt = torch.float32 if f32.value else torch.float64
        disp = self._view(dd.value, dim * Nl * self.S * (4 if f32.value else 8), dt, (dim, Nl, self.S))
        sig = None
        if ds.value:
            sig = self._view(ds.value, dim * Nl * self.S * 8, torch.float64, (dim, Nl, self.S))
        return disp, sig

    def autotune(self, cache_path=None, stream=None):
        """Pick the level-0 launch shape by timing (slm_autotune); with a
        cache file the choice is read from / appended to it."""
        cp = None if cache_path is None else str(cache_path).encode()
        N.check(N.lib().slm_autotune(self.h, None, 0, cp, _stream(stream)), self.h)
        return self

    def tile_choice(self):
        """The 2D level-0 tile shape index in force (slm_launch_info), or
        None when the level-0 step is not LDS-tiled."""
        t, _ = self.launch_info(0, max(1, self.N[0] // max(1, self.m[0])))
        return t - 1 if t > 0 else None

    def launch_info(self, level, nchains):
        """(tiled, blocks_per_system) of level ``level``'s step over
        ``nchains`` intervals (slm_launch_info)."""
        t, b = C.c_int(), C.c_int()
        N.check(N.lib().slm_launch_info(self.h, level, nchains, C.byref(t), C.byref(b)), self.h)
        return t.value, b.value

    # ------------------------------------------------------------ operators
    def _dev(self, x):
        x = torch.as_tensor(x)
        return x.to(device=self.device, dtype=self.dtype).contiguous()

    def apply_phi(self, level, n0, x, stream=None):
        """out[k] = Phi_level(n0+k) x[k]; x is [count][S]."""
        x = self._dev(x).reshape(-1, self.S)
        out = torch.empty_like(x)
        N.check(N.lib().slm_apply_phi(self.h, level, n0, x.shape[0], _ptr(x), _ptr(out), _stream(stream)), self.h)
        return out

    def relax(self, level, mode, c_in=None, g=None, stream=None):
        """One batched relaxation sweep (see slm_relax).  Returns the
        tensor(s) the sweep writes."""
        Nl, m = self.N[level], self.m[level]
        nc = Nl // m
        cin = None if c_in is None else self._dev(c_in).reshape(nc + 1, self.S)
        gg = None if g is None else self._dev(g).reshape(Nl + 1, self.S)
        cout = res = v = None
        norm = C.c_double(0.0)
        if mode == "FC":
            cout = torch.zeros(nc + 1, self.S, dtype=self.dtype, device=self.device)
        elif mode == "RES":
            res = torch.zeros(nc + 1, self.S, dtype=self.dtype, device=self.device)
        else:
            v = torch.zeros(Nl + 1, self.S, dtype=self.dtype, device=self.device)
        N.check(N.lib().slm_relax(self.h, level, N.SWEEP[mode], _ptr(gg), _ptr(cin), _ptr(cout), _ptr(res),
                                  _ptr(v), C.byref(norm), _stream(stream)), self.h)
        if mode == "FC":
            return cout
        if mode == "RES":
            return res, norm.value
        return v

    def relax_into(self, level, mode, c_in=None, g=None, c_out=None, res=None, v=None, stream=None):
        """slm_relax on preallocated device tensors (no allocation; for timing)."""
        N.check(N.lib().slm_relax(self.h, level, N.SWEEP[mode], _ptr(g), _ptr(c_in), _ptr(c_out), _ptr(res),
                                  _ptr(v), None, _stream(stream)), self.h)

    def step(self, u0, store_all=True, stream=None):
        u0 = self._dev(u0).reshape(self.S)
        shape = (self.pr.nt + 1, self.S) if store_all else (self.S,)
        u = torch.empty(shape, dtype=self.dtype, device=self.device)
        N.check(N.lib().slm_step(self.h, _ptr(u0), _ptr(u), int(store_all), _stream(stream)), self.h)
        return u

    def seed_iterate(self, u, seed, cpoints=False, stream=None):
        """Write the seeded initial iterate (slm_seed_iterate) into the
        C-points of ``u``: [nt+1][S] (``cpoints=False``) or [nt/m0+1][S]."""
        assert u.dtype == self.dtype and u.is_contiguous()
        N.check(N.lib().slm_seed_iterate(self.h, C.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), _ptr(u), int(bool(cpoints)),
                                         _stream(stream)), self.h)
        return u

    def solve(self, u0, u, hist_cap=512, stream=None):
        """MGRIT in place on ``u`` ([nt+1][S] device tensor whose C-points are
        the initial iterate).  Returns (stats dict, residual history)."""
        assert u.dtype == self.dtype and u.is_contiguous() and u.numel() == (self.pr.nt + 1) * self.S
        u0 = self._dev(u0).reshape(self.S)
        st = N.Stats()
        hist = (C.c_double * hist_cap)()
        rc = N.lib().slm_solve(self.h, _ptr(u0), _ptr(u), C.byref(st), hist, hist_cap, _stream(stream))
        N.check(rc, self.h)
        stats = _stats_dict(st)
        nh = min(hist_cap, st.iterations)
        return stats, np.array([hist[i] for i in range(nh)])

    @property
    def n_cpoints(self):
        return self.pr.nt // self.m[0] + 1

    def solve_cpoints(self, u0, c, hist_cap=512, stream=None):
        """MGRIT keeping only the C-points: ``c`` ([nt/m0+1][S] device tensor)
        holds the initial iterate on entry and the converged C-values on
        exit.  Returns (stats, history)."""
        assert c.dtype == self.dtype and c.is_contiguous() and c.numel() == self.n_cpoints * self.S
        u0 = self._dev(u0).reshape(self.S)
        st = N.Stats()
        hist = (C.c_double * hist_cap)()
        N.check(N.lib().slm_solve_cpoints(self.h, _ptr(u0), _ptr(c), C.byref(st), hist, hist_cap,
                                          _stream(stream)), self.h)
        return _stats_dict(st), np.array([hist[i] for i in range(min(hist_cap, st.iterations))])

    def adjoint(self, c, lamT, hist_cap=512, stream=None):
        """Gradient of a final-time misfit with dL/du_nt = ``lamT``, from the
        C-point checkpoints ``c``.  Returns (dL/du0 device tensor, dL/dtheta
        numpy array [n_alpha + n_beta], stats, history)."""
        lamT = self._dev(lamT).reshape(self.S)
        g0 = torch.empty(self.S, dtype=torch.float64, device=self.device)
        nq = len(self.pr.alpha) + (len(self.pr.beta or []) if self.pr.dim == 2 else 0)
        gth = (C.c_double * max(1, nq))()
        st = N.Stats()
        hist = (C.c_double * hist_cap)()
        N.check(N.lib().slm_adjoint(self.h, _ptr(c), _ptr(lamT), _ptr(g0), gth, C.byref(st), hist, hist_cap,
                                    _stream(stream)), self.h)
        return (g0, np.array([gth[q] for q in range(nq)]), _stats_dict(st),
                np.array([hist[i] for i in range(min(hist_cap, st.iterations))]))


def _stats_dict(st):
    return dict(iterations=st.iterations, status=N.STATUS.get(st.status, str(st.status)),
                n_levels=st.n_levels, rho0=st.rho0, rho_final=st.rho_final, solve_ms=st.solve_ms,
                point_updates=st.point_updates, gmres_solves=st.gmres_solves, gmres_iters=st.gmres_iters)


class Batch:
    """Many independent 1D problems (a list of ``(Problem, Solver)``) solved
    together by the batched V-cycle of ``slm_batch_solve``."""

    def __init__(self, problems, precision="fp64", device="cuda"):
        if torch is None:
            raise N.NativeError("torch is required for device memory")
        self.problems = list(problems)
        self.n = len(self.problems)
        self.precision = precision
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        descs = (N.Desc * max(1, self.n))()
        self._keep = []
        for i, (pr, sv) in enumerate(self.problems):
            d, k = N.make_desc(pr, sv, precision)
            descs[i] = d
            self._keep.append(k)
        self._descs = descs
        h = C.c_void_p()
        N.check(N.lib().slm_batch_create(descs, self.n, C.byref(h)))
        self.h = h
        nb = C.c_size_t()
        N.check(N.lib().slm_batch_workspace_size(self.h, C.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                N.lib().slm_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def setup(self, stream=None):
        if self.ws is None:
            self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws_raw.data_ptr()) % 256
            self.ws = self._ws_raw[off:off + self.ws_bytes]
        N.check(N.lib().slm_batch_setup(self.h, _ptr(self.ws), self.ws_bytes, _stream(stream)))
        return self

    def tune(self, cache_path=None, stream=None):
        cp = None if cache_path is None else str(cache_path).encode()
        N.check(N.lib().slm_batch_tune(self.h, cp, _stream(stream)))
        return self

    def solve(self, u0s, us, use_graph=True, hist_cap=512, stream=None):
        """Solve every problem in place on ``us[i]`` ([nt_i+1][nx_i] device
        tensors whose C-points are the initial iterates); ``u0s[i]`` are the
        initial conditions.  Returns (list of stats dicts, list of histories)."""
        assert len(u0s) == self.n and len(us) == self.n
        u0d = []
        for i, (pr, _) in enumerate(self.problems):
            assert us[i].dtype == self.dtype and us[i].is_contiguous() and us[i].numel() == (pr.nt + 1) * pr.nx
            u0d.append(torch.as_tensor(u0s[i]).to(device=self.device, dtype=self.dtype).contiguous().reshape(pr.nx))
        a0 = (C.c_void_p * self.n)(*[t.data_ptr() for t in u0d])
        a1 = (C.c_void_p * self.n)(*[t.data_ptr() for t in us])
        st = (N.Stats * self.n)()
        hist = (C.c_double * (self.n * hist_cap))()
        rc = N.lib().slm_batch_solve(self.h, a0, a1, st, hist, hist_cap, int(bool(use_graph)), _stream(stream))
        N.check(rc)
        stats = [_stats_dict(st[i]) for i in range(self.n)]
        hs = [np.array([hist[i * hist_cap + k] for k in range(min(hist_cap, stats[i]["iterations"]))])
              for i in range(self.n)]
        return stats, hs
