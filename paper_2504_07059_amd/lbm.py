"""Python face of the HIP library: argument marshalling only.  torch supplies
device memory and the stream; every step of the method runs in the library's
kernels."""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Params, check, lib


def make_params(lattice, nx, ny, nz, masses, diff, tau1, g=(0.0, 0.0, 0.0),
                walls=(False, False, False), n0=0.0, forcing=0, wall_velocity=None,
                wall_kind="appendix_a"):
    """Fill one lbm_mc_params struct (forcing: 0 or "standard" for the
    standard forcing term, 1 or "diff" to add the diffusion-driven term, 2 or
    "full" for the whole corrected forcing, - S_p + S_rho + S_diff;
    wall_velocity: optional [[low], [high]] tangential velocities of the two
    walls of the wall axis; wall_kind: "appendix_a" for the impermeable walls
    of Appendix A, "equilibrium" for the comparison boundary of Sec. 4.1)."""
    p = Params()
    p.lattice = {"D2Q9": _lib.D2Q9, "D3Q19": _lib.D3Q19}[lattice] if isinstance(lattice, str) \
        else int(lattice)
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    N = len(masses)
    p.n_species = N
    for a in range(3):
        p.bc[a] = ({"appendix_a": _lib.WALL, "equilibrium": _lib.WALL_EQ}[wall_kind]
                   if walls[a] else _lib.PERIODIC)
    for i in range(N):
        p.molar_mass[i] = float(masses[i])
        for j in range(N):
            p.diff[i][j] = float(diff[i][j]) if i != j else 0.0
    p.tau1 = float(tau1)
    for a in range(3):
        p.g[a] = float(g[a])
    p.n0 = float(n0 or 0.0)
    p.forcing = {"standard": 0, "diff": 1, "full": 2}[forcing] if isinstance(forcing, str) \
        else int(forcing)
    p.reserved = 0
    for k in range(2):
        for a in range(3):
            p.wall_velocity[k][a] = float(wall_velocity[k][a]) if wall_velocity is not None else 0.0
    return p


def params_from_workload(w):
    return make_params(w.lattice, w.nx, w.ny, w.nz, w.masses, w.diff, w.tau1, w.g,
                       w.walls, w.n0 or 0.0, w.forcing, w.wall_velocity, w.wall_kind)


def _arr(params):
    if isinstance(params, Params):
        params = [params]
    arr = (Params * len(params))(*params)
    return arr, len(params)


def layout(params):
    arr, L = _arr(params)
    total = ctypes.c_int64()
    offs = (ctypes.c_int64 * L)()
    pitch = (ctypes.c_int32 * L)()
    fields = (ctypes.c_int64 * L)()
    check(lib.lbm_mc_layout(arr, L, ctypes.byref(total), offs, pitch, fields))
    return total.value, list(offs), list(pitch), list(fields)


def check_problem(params, x0):
    arr, L = _arr(params)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    lam = ctypes.c_double()
    st = lib.lbm_mc_check(arr, L, x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          ctypes.byref(lam))
    return st, lam.value, lib.lbm_mc_last_error().decode()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class LbmMc:
    """One context of the library over torch-owned population buffers.

    params: one Params or a list (batched); x0: float64 array [L*N*nodes]
    (or any array whose C-order flattening is that).  accel: optional force
    field k(x) replacing g (params' g must be 0), float32 on the device,
    [d, nz, ny, nx] per lattice concatenated (d = 2 or 3); kept referenced
    by the context, which reads it every step."""

    def __init__(self, params, x0, device="cuda", stream=None, accel=None):
        self._arr, self.L = _arr(params)
        self.params = list(self._arr)
        self.total, self.offsets, self.pitch, self.field_offsets = layout(self.params)
        self.N = self.params[0].n_species
        self.lattice = self.params[0].lattice
        self.Q = 9 if self.lattice == _lib.D2Q9 else 19
        self.dim = 2 if self.lattice == _lib.D2Q9 else 3
        self.nodes = [p.nx * p.ny * p.nz for p in self.params]
        self.device = torch.device(device)
        self.fa = torch.empty(self.total, dtype=torch.float32, device=self.device)
        self.fb = torch.empty(self.total, dtype=torch.float32, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(-1))
        self._x0 = x0
        self.ctx = ctypes.c_void_p()
        xp = x0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        if accel is None:
            self.accel = None
            check(lib.lbm_mc_init(self._arr, self.L, xp, _ptr(self.fa), _ptr(self.fb),
                                  self.total, sp, ctypes.byref(self.ctx)))
        else:
            want = self.dim * sum(self.nodes)
            if accel.dtype != torch.float32 or accel.device != self.fa.device or \
                    accel.numel() != want:
                raise ValueError(f"accel must be float32 on {self.fa.device} with {want} values")
            self.accel = accel.contiguous()
            check(lib.lbm_mc_init_field(self._arr, self.L, xp, _ptr(self.accel), _ptr(self.fa),
                                        _ptr(self.fb), self.total, sp, ctypes.byref(self.ctx)))

    # ---------------------------------------------------------------- stepping
    def step(self, n=1):
        check(lib.lbm_mc_step(self.ctx, int(n)))

    def prepare(self, n):
        """Capture ahead of time the step graphs that step(n) will replay."""
        check(lib.lbm_mc_prepare(self.ctx, int(n)))

    def sync(self):
        check(lib.lbm_mc_sync(self.ctx))

    @property
    def t(self):
        t = ctypes.c_int64()
        check(lib.lbm_mc_state(self.ctx, None, None, ctypes.byref(t)))
        return t.value

    def buffers(self):
        """(cur, prev) torch views: f~(t) and f~(t-1)."""
        cur, prev = ctypes.c_void_p(), ctypes.c_void_p()
        check(lib.lbm_mc_state(self.ctx, ctypes.byref(cur), ctypes.byref(prev), None))
        a = self.fa if cur.value == self.fa.data_ptr() else self.fb
        b = self.fb if a is self.fa else self.fa
        return a, b

    def raw(self, which="cur", lattice=0):
        """[N, Q, nz, ny, nx] view of one lattice's stored state: plane 0 of a
        species is its rest population P0 = f~_0, plane a >= 1 is
        g_a = f~_a - (w_a/w_0) P0."""
        buf = self.buffers()[0 if which == "cur" else 1]
        p = self.params[lattice]
        n = self.N * self.Q * p.nz * p.ny * self.pitch[lattice]
        v = buf[self.offsets[lattice]: self.offsets[lattice] + n]
        return v.view(self.N, self.Q, p.nz, p.ny, self.pitch[lattice])[..., : p.nx]

    def moments(self, fields=True, velocities=False):
        """Observables of f(t): dict with 'rho', 'x' [sum_l N*nodes], 'u'
        [sum_l dim*nodes] (device tensors), with velocities also 'ueq' and
        'us' [sum_l N*dim*nodes] (u_i^eq and the real species velocity u_i),
        and 'mass' [L, N], 'momentum' [L, dim] (numpy float64)."""
        tot = sum(self.nodes)
        out = {}
        f32 = dict(dtype=torch.float32, device=self.device)
        if fields:
            out["rho"] = torch.empty(tot * self.N, **f32)
            out["x"] = torch.empty(tot * self.N, **f32)
            out["u"] = torch.empty(tot * self.dim, **f32)
        if velocities:
            out["ueq"] = torch.empty(tot * self.N * self.dim, **f32)
            out["us"] = torch.empty(tot * self.N * self.dim, **f32)
        mass = np.zeros((self.L, self.N))
        mom = np.zeros((self.L, self.dim))
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib.lbm_mc_moments(self.ctx, _ptr(out.get("rho")), _ptr(out.get("x")),
                                 _ptr(out.get("u")), _ptr(out.get("ueq")), _ptr(out.get("us")),
                                 mass.ctypes.data_as(dp), mom.ctypes.data_as(dp)))
        out["mass"] = mass
        out["momentum"] = mom
        return out

    def field(self, out, name, lattice=0):
        """Reshape a node field of `moments()` for one lattice: [k, nz, ny, nx]
        ('rho', 'x': k = N; 'u': k = dim), or [N, dim, nz, ny, nx] ('ueq', 'us')."""
        p = self.params[lattice]
        k = {"rho": self.N, "x": self.N, "u": self.dim}.get(name, self.N * self.dim)
        off = self.field_offsets[lattice] * k
        n = self.nodes[lattice] * k
        v = out[name][off: off + n]
        if name in ("ueq", "us"):
            return v.view(self.N, self.dim, p.nz, p.ny, p.nx)
        return v.view(k, p.nz, p.ny, p.nx)

    def restore(self, cur, prev, t):
        check(lib.lbm_mc_restore(self.ctx, _ptr(cur), _ptr(prev), int(t)))

    # ------------------------------------------------------------------ tuning
    def set_tuning(self, block_x=0, block_y=0, rows=0, persistent=-1, variant=-1):
        check(lib.lbm_mc_set_tuning(self.ctx, block_x, block_y, rows, persistent, variant))

    def get_tuning(self):
        """(block_x, block_y, rows, persistent, variant)."""
        v = [ctypes.c_int32() for _ in range(5)]
        check(lib.lbm_mc_get_tuning(self.ctx, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def autotune(self, reps=5):
        """Pick the fastest execution shape.  Invalidates f~(t-1); callers that
        need moments right away should build a fresh context (the choice is
        cached for the process)."""
        best = ctypes.c_double()
        check(lib.lbm_mc_autotune(self.ctx, int(reps), ctypes.byref(best)))
        return best.value

    def set_batched_mode(self, one_launch):
        check(lib.lbm_mc_set_batched_mode(self.ctx, int(one_launch)))

    # ----------------------------------------------------------------- adjoint
    def view(self, buf, lattice=0):
        """[N, Q, nz, ny, nx] view of one lattice inside any flat buffer of the
        population layout (a state, an adjoint field)."""
        p = self.params[lattice]
        n = self.N * self.Q * p.nz * p.ny * self.pitch[lattice]
        v = buf[self.offsets[lattice]: self.offsets[lattice] + n]
        return v.view(self.N, self.Q, p.nz, p.ny, self.pitch[lattice])[..., : p.nx]

    # ----------------------------------------------------------------- adjoint
    def adjoint_step(self, f_prev, lam_in, lam_out, grad):
        check(lib.lbm_mc_adjoint_step(self.ctx, _ptr(f_prev), _ptr(lam_in), _ptr(lam_out),
                                      _ptr(grad)))

    def adjoint_init(self, lam0, grad):
        check(lib.lbm_mc_adjoint_init(self.ctx, _ptr(lam0), _ptr(grad)))

    def replay(self, src, n, states):
        """states: [>= n, stride] float32 rows; row k <- the state k+1 steps after src."""
        check(lib.lbm_mc_replay(self.ctx, _ptr(src), int(n), _ptr(states), states.stride(0)))

    def adjoint_run(self, states, n, lam_in, lam_out, grad):
        """Reverse n steps through rows 0..n-1 of states (= s(t0) .. s(t0+n-1))."""
        check(lib.lbm_mc_adjoint_run(self.ctx, _ptr(states), states.stride(0), int(n),
                                     _ptr(lam_in), _ptr(lam_out), _ptr(grad)))

    # ---------------------------------------------------------------- profile
    def profile(self, state=None, out=None):
        """Mole-fraction profile along x, averaged over y and z, of a stored
        state (default: the current buffer): float64 [N, nx] on the device."""
        state = self.buffers()[0] if state is None else state
        p = self.params[0]
        if out is None:
            out = torch.empty((self.N, p.nx), dtype=torch.float64, device=self.device)
        check(lib.lbm_mc_profile(self.ctx, _ptr(state), _ptr(out)))
        return out

    def profile_static(self, state=None, out=None):
        """profile() through the allocation-free entry point (its partial sums
        in the library's fixed device array)."""
        state = self.buffers()[0] if state is None else state
        p = self.params[0]
        if out is None:
            out = torch.empty((self.N, p.nx), dtype=torch.float64, device=self.device)
        check(lib.lbm_mc_profile_static(self.ctx, _ptr(state), _ptr(out)))
        return out

    def profile_vjp(self, state, dxbar, lam):
        """lam <- (d profile / d state)^T dxbar (dxbar float64 [N, nx] on the
        device; lam a float32 buffer of the population layout)."""
        dxbar = dxbar.to(device=self.device, dtype=torch.float64).contiguous()
        check(lib.lbm_mc_profile_vjp(self.ctx, _ptr(state), _ptr(dxbar), _ptr(lam)))

    def close(self):
        if self.ctx:
            lib.lbm_mc_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
