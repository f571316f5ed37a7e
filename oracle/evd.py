"""The EVD multicomponent LBM with forcing, written plainly in torch float64.

Lattice units throughout: delta_x = delta_t = 1 (Sec. 4 opening).
Population tensors have shape [N, Q, nz, ny, nx] (species, direction, z, y, x);
2-D lattices use nz = 1.  Species are ordered by ascending molar mass and the
masses are normalised so that M_1 = 1, hence c_1 = 1 (Sec. 4 opening).

One time step is  f(t) --collide--> f~(t) --stream + walls--> f(t+1):
  * collide: eq. (LBE_forcing) with Omega = Omega^ii + sum_j Omega^ij
    (eqs. BGK_self_collision, Cross_collision_Sirovich), the equilibria of
    eq. (feqi0) and the one after it, and the standard forcing term of
    eq. (CE_forcing_term_discretized); the moments entering them are eqs.
    (zeroth_order_moment), (first_order_moment_force), (Sirovich_mixture_density)
    and (Sirovich_mixture_velocity); tau_ij solves eq. (relation_tauij_diff_coeff)
    at every node (Sec. 4.1).
  * stream: eq. (Second_order_spatial_interpolation), read as quadratic Lagrange
    interpolation of the post-collision values of the 3x3 (3x3x3) neighbourhood
    at the departure point, then the impermeable-wall scheme of Appendix A.

Readings taken where the paper is silent (each repeated at its function):
  R1 the primed points of the interpolation formula are the landing positions
     of the neighbours' post-collision populations, with A = (+1,0), B = (0,+1),
     C = (-1,0), D = (0,-1), E = (+1,+1), F = (-1,+1), G = (-1,-1), H = (+1,-1)
     as source offsets from the target O (the only labelling under which c = 1
     is an exact shift and Appendix A's right wall has its solid node at A);
  R2 the wall scheme of Appendix A, stated per wall and per direction there,
     is applied as one rule for any single wall axis, 2-D or 3-D;
  R3 for N > 3 species the tau relation is solved with the index convention of
     the paper's ternary solution: for the pair i < j the sum runs over
     rho_s / tau_sj;
  R4 a species with rho_i = 0 at a node takes u_i^eq = F_i/(2 rho_i) -> k_i/2
     (any finite value gives the same populations, as everything it enters is
     multiplied by rho_i);
  R5 pressure p = n M_1 c_{s,1}^2 with c_{s,1}^2 = 1/3 (standard D2Q9 value);
  R6 the gradients in the pressure and density forcing contributions of
     eq. (improved_forcing_scheme) are taken from the densities of the
     streamed populations at the same time level, by second-order central
     differences along each lattice axis (periodic axes wrap); at a node next
     to a wall the second-order one-sided difference into the fluid is used
     (a wall axis then needs at least 3 nodes);
  R11 where walls on several axes meet (edges, corners; Appendix A treats
     single walls), the wall rule is read as the return, to the wall node,
     of what its populations would stream beyond the walls, split by the set
     of walls crossed (see _wall_returns); it reduces to Appendix A for one
     wall, to halfway bounce-back at c = 1, and conserves mass;
  R12 the real species velocity of a species with rho_i = 0 at a node (eq.
     CE_EQ83 divides Theta_i by rho_i) is the limit rho_i -> 0, in which
     Theta_i/rho_i = sum_j rho_j/(rho tau_ij)(u_i^eq - u_j^eq);
  R10 the moving-wall term of Appendix A takes rho_i and the mass fraction
     w_i of the streamed populations at the wall node (the term adds no mass,
     so they do not depend on it), and a wall moves only along itself.
"""
import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

from .lattice import Lattice, DTYPE

AXIS_DIM = {0: -1, 1: -2, 2: -3}   # x, y, z -> spatial tensor dimension


def lagrange_weights(s):
    """1-D weights (lambda_-1, lambda_0, lambda_+1) of the source nodes at
    offsets -1, 0, +1 from the target, for Courant number s.

    They are the one-dimensional factors of eq. (Second_order_spatial_
    interpolation): the coefficient of C' is xi(1+xi)/2, of O' is 1-xi^2 and of
    A' is -xi(1-xi)/2 (reading R1)."""
    return (s * (1.0 + s) / 2.0, 1.0 - s * s, -s * (1.0 - s) / 2.0)


@dataclass
class Model:
    """Problem statement of the method (Sec. 4.1 and 4.2): lattice, species
    molar masses, pair diffusivities D_ij (lattice units), tau_1 (viscosity),
    specific body force k (F_i = rho_i k, eq. MS_equation), and per-axis
    impermeable walls (Appendix A) or periodicity."""
    lattice: str
    nx: int
    ny: int
    nz: int
    masses: Sequence[float]
    diff: torch.Tensor                  # [N, N] symmetric, lattice units
    tau1: float
    g: torch.Tensor = None              # [3] specific force (gravity)
    walls: Sequence[bool] = (False, False, False)
    n0: Optional[float] = None
    force_field: Optional[torch.Tensor] = None   # [3, nz, ny, nx] overrides g
    wall_velocity: Optional[torch.Tensor] = None # [2, 3]: velocity of the wall at the low
                                                 # and high end of the wall axis (tangential)
    forcing: str = "standard"   # "standard": eq. (CE_forcing_term_discretized);
                                # "diff": plus S_diff of eq. (improved_forcing_scheme);
                                # "full": the whole of eq. (improved_forcing_scheme),
                                # i.e. - S_p + S_rho + S_diff

    def __post_init__(self):
        self.lat = Lattice(self.lattice)
        self.N = len(self.masses)
        if list(self.masses) != sorted(self.masses):
            raise ValueError("species must be ordered by ascending molar mass")
        m1 = float(self.masses[0])
        # Sec. 4 opening: M_1 = 1 for the lightest species.
        self.M = [float(m) / m1 for m in self.masses]
        self.diff = torch.as_tensor(self.diff, dtype=DTYPE)
        if self.g is None:
            self.g = torch.zeros(3, dtype=DTYPE)
        self.g = torch.as_tensor(self.g, dtype=DTYPE)
        if self.lat.dim == 2 and self.nz != 1:
            raise ValueError("2-D lattice needs nz = 1")

        for a, w in enumerate(self.walls):
            if w and self.shape_axis(a) < 2:
                raise ValueError("a wall axis needs at least 2 nodes")
        if self.lat.dim == 2 and self.walls[2]:
            raise ValueError("no z walls in 2-D")
        if self.wall_velocity is not None:
            self.wall_velocity = torch.as_tensor(self.wall_velocity, dtype=DTYPE)
            ax = [a for a in range(3) if self.walls[a]]
            if not ax:
                raise ValueError("a wall velocity needs a wall axis")
            if len(ax) > 1:
                raise ValueError("moving walls need a single wall axis")
            if bool((self.wall_velocity[:, ax[0]] != 0).any()):
                raise ValueError("wall velocities must be tangential to the wall")
            if self.lat.dim == 2 and bool((self.wall_velocity[:, 2] != 0).any()):
                raise ValueError("no z velocity in 2-D")
        if self.forcing not in ("standard", "diff", "full"):
            raise ValueError("forcing must be 'standard', 'diff' or 'full'")
        if self.forcing == "full":
            for a in range(3):
                if self.walls[a] and self.shape_axis(a) < 3:
                    raise ValueError("the full forcing needs >= 3 nodes on a wall axis")

    def shape_axis(self, a):
        return (self.nx, self.ny, self.nz)[a]

    # ---------------------------------------------------------------- S0
    def speeds(self):
        """c_i = sqrt(M_1/M_i), eq. (speed_DLS) with c_1 = 1."""
        return [math.sqrt(1.0 / m) for m in self.M]

    def sound2(self):
        """c_{s,i}^2 = c_i^2 / 3 (reading R5 applied per species via eq. speed_DLS)."""
        return [c * c / 3.0 for c in self.speeds()]

    def taus(self):
        """tau_i from nu_i = (tau_i - 1/2) c_{s,i}^2 equal for all species
        (Sec. 3, after eq. epecies_momentum_eq; Sec. 4 opening)."""
        return [0.5 + (self.tau1 - 0.5) * m for m in self.M]

    def velocities(self):
        """e^i_alpha = c_i * integer direction, eq. (discrete_velocity_DLS).
        Returns [N, Q, 3]."""
        c = torch.tensor(self.speeds(), dtype=DTYPE)
        return c[:, None, None] * self.lat.c[None, :, :]

    def accel(self):
        """Specific force k at every node, [3, nz, ny, nx]."""
        if self.force_field is not None:
            return self.force_field.to(DTYPE)
        return self.g[:, None, None, None].expand(3, self.nz, self.ny, self.nx)

    def default_n0(self):
        """Total mole number of the initial state: n = sum_i x_i rho_i0 / M_i
        (Sec. 4.1) with ideal pure densities rho_i0 = M_i / M_max, i.e. the
        heaviest pure species has rho = 1 (Sec. 4 opening).  Then n = 1/M_max
        whatever the composition."""
        return 1.0 / max(self.M) if self.n0 is None else float(self.n0)


def _dot(a, b):
    """Sum over the last component axis of [..., 3]-shaped factors."""
    return (a * b).sum(dim=-1)


# -------------------------------------------------------------------- moments
def species_moments(model, f):
    """rho_i (eq. zeroth_order_moment) and u_i^eq with the force shift
    (eq. first_order_moment_force):  u_i^eq = (sum_a e f)/rho_i + F_i/(2 rho_i),
    F_i = rho_i k.  Reading R4 for rho_i = 0.

    Returns rho [N, nz, ny, nx] and ueq [N, nz, ny, nx, 3]."""
    e = model.velocities()                                 # [N, Q, 3]
    rho = f.sum(dim=1)
    mom = torch.einsum("nqc,nqzyx->nzyxc", e, f)
    k = model.accel().permute(1, 2, 3, 0)[None]            # [1, nz, ny, nx, 3]
    safe = torch.where(rho == 0, torch.ones_like(rho), rho)
    ueq = torch.where((rho == 0)[..., None], 0.5 * k.expand_as(mom),
                      mom / safe[..., None] + 0.5 * k)
    return rho, ueq


def mixture(model, rho_i, ueq):
    """rho = sum rho_i (eq. Sirovich_mixture_density),
    u = sum w_i u_i^eq with w_i = rho_i/rho (eq. Sirovich_mixture_velocity),
    n = sum rho_i/M_i (Sec. 3, after eq. CE_EQ102) and p = n M_1 c_{s,1}^2
    (Sec. 4.1, reading R5)."""
    rho = rho_i.sum(dim=0)
    w = rho_i / rho
    u = (w[..., None] * ueq).sum(dim=0)
    M = torch.tensor(model.M, dtype=DTYPE)
    n = (rho_i / M[:, None, None, None]).sum(dim=0)
    p = n * model.M[0] * model.sound2()[0]
    return rho, u, n, p


def cross_relaxation(model, rho_i, rho, n, p):
    """Inverse cross-relaxation times y_ij = 1/tau_ij at every node, from
    eq. (relation_tauij_diff_coeff):

      [(rho_i+rho_j)/D_ij + 2 n^2 M_i M_j/(p dt)] y_ij
          + (1/D_ij) sum_{s != i,j} rho_s y_sj  =  2 rho/(D_ij dt)

    with the index convention of the ternary solution of Sec. 4.1 (reading R3):
    the unknowns of the pairs (i, j), i < j, that share the larger index j form
    one dense linear system once the y_js with s > j are known, so the columns
    are solved for j = N, N-1, ..., 2 with a library solver.

    Returns Y [N, N, nz, ny, nx], symmetric, zero diagonal."""
    N = model.N
    D = model.diff
    M = model.M
    shape = rho.shape
    P = rho.numel()
    r = rho_i.reshape(N, P)
    R = rho.reshape(P)
    nn = n.reshape(P)
    pp = p.reshape(P)
    Y = [[None] * N for _ in range(N)]
    zero = torch.zeros(P, dtype=DTYPE)
    for j in range(N - 1, 0, -1):
        rows = list(range(j))
        A = torch.zeros(P, j, j, dtype=DTYPE)
        b = torch.zeros(P, j, dtype=DTYPE)
        for ii, i in enumerate(rows):
            Dij = D[i, j]
            A_ij = (r[i] + r[j]) / Dij + 2.0 * nn * nn * M[i] * M[j] / pp
            for kk, s in enumerate(rows):
                if s == i:
                    A[:, ii, kk] = A_ij
                else:
                    A[:, ii, kk] = r[s] / Dij
            known = zero
            for s in range(j + 1, N):
                known = known + r[s] * Y[j][s]
            b[:, ii] = 2.0 * R / Dij - known / Dij
        y = torch.linalg.solve(A, b)
        for ii, i in enumerate(rows):
            Y[i][j] = y[:, ii]
            Y[j][i] = y[:, ii]
    for i in range(N):
        Y[i][i] = zero
    out = torch.stack([torch.stack(row) for row in Y])
    return out.reshape(N, N, *shape)


# -------------------------------------------------------------------- collide
def equilibria(model, rho_i, ueq, u):
    """f^(eq) (second-order Hermite form in the mixture velocity u) and
    f^(0) = [1 + (e - u).(u_i^eq - u)/c_s^2] f^(eq), eq. (feqi0) and the
    equation after it.  Returns two tensors [N, Q, nz, ny, nx]."""
    e = model.velocities()
    w = model.lat.w
    cs2 = torch.tensor(model.sound2(), dtype=DTYPE)[:, None, None, None, None]
    eu = torch.einsum("nqc,zyxc->nqzyx", e, u)
    uu = _dot(u, u)[None, None]
    feq = w[None, :, None, None, None] * rho_i[:, None] * (
        1.0 + eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2))
    du = ueq - u[None]                                     # [N, nz, ny, nx, 3]
    e_du = torch.einsum("nqc,nzyxc->nqzyx", e, du)
    u_du = _dot(u[None], du)[:, None]
    f0 = (1.0 + (e_du - u_du) / cs2) * feq
    return feq, f0


def forcing_term(model, rho_i, u):
    """Standard forcing term, eq. (CE_forcing_term_discretized):
    S = omega [ e/c_s^2 + (e e - c_s^2 I).u / c_s^4 ] . F_i,  F_i = rho_i k."""
    e = model.velocities()
    w = model.lat.w
    cs2 = torch.tensor(model.sound2(), dtype=DTYPE)[:, None, None, None, None]
    k = model.accel().permute(1, 2, 3, 0)                  # [nz, ny, nx, 3]
    F = rho_i[..., None] * k[None]                         # [N, nz, ny, nx, 3]
    eF = torch.einsum("nqc,nzyxc->nqzyx", e, F)
    eu = torch.einsum("nqc,zyxc->nqzyx", e, u)
    uF = _dot(u[None], F)[:, None]
    # [e/c2 + (e (e.u) - c2 u)/c2^2] . F
    S = eF / cs2 + (eu * eF - cs2 * uF) / (cs2 * cs2)
    return w[None, :, None, None, None] * S


def theta(model, rho_i, rho, ueq, Y):
    """Theta_i = sum_j (rho_i rho_j / (rho tau_ij)) (u_i^eq - u_j^eq), the
    momentum the velocity-difference relaxation removes from species i
    (eq. CE_theta_definition).  [N, nz, ny, nx, 3]."""
    N = model.N
    out = torch.zeros_like(ueq)
    for i in range(N):
        for j in range(N):
            if i != j:
                out[i] = out[i] + (rho_i[i] * rho_i[j] / rho * Y[i, j])[..., None] \
                    * (ueq[i] - ueq[j])
    return out


def theta_per_density(model, rho_i, rho, ueq, Y):
    """Theta_i / rho_i = sum_j (rho_j / (rho tau_ij)) (u_i^eq - u_j^eq), from
    eq. (CE_theta_definition) with the common factor rho_i cancelled; where
    rho_i = 0 this is the limit of Theta_i/rho_i (reading R12).
    [N, nz, ny, nx, 3]."""
    N = model.N
    out = torch.zeros_like(ueq)
    for i in range(N):
        for j in range(N):
            if i != j:
                out[i] = out[i] + (rho_i[j] / rho * Y[i, j])[..., None] * (ueq[i] - ueq[j])
    return out


def diffusion_forcing(model, th, u):
    """Diffusion-driven forcing contribution of eq. (improved_forcing_scheme):
    S_diff = omega (dt/(2 tau_i - dt)) [(e e - c_s^2 I)/c_s^4 . u] . Theta_i,
    i.e. omega/(2 tau_i - 1) [(e.u)(e.Theta_i) - c_s^2 u.Theta_i]/c_s^4 (dt = 1)."""
    e = model.velocities()
    w = model.lat.w
    cs2 = torch.tensor(model.sound2(), dtype=DTYPE)[:, None, None, None, None]
    tau = torch.tensor(model.taus(), dtype=DTYPE)[:, None, None, None, None]
    eu = torch.einsum("nqc,zyxc->nqzyx", e, u)
    eth = torch.einsum("nqc,nzyxc->nqzyx", e, th)
    uth = _dot(u[None], th)[:, None]
    return w[None, :, None, None, None] / (2.0 * tau - 1.0) * (eu * eth - cs2 * uth) / (cs2 * cs2)


def gradient(model, phi):
    """Discrete gradient of a node field phi [nz, ny, nx] (reading R6):
    (phi(x+1) - phi(x-1))/2 along each lattice axis, wrapped on periodic
    axes; on a wall axis the first and last nodes take the one-sided
    differences (-3 phi_0 + 4 phi_1 - phi_2)/2 and
    (3 phi_{n-1} - 4 phi_{n-2} + phi_{n-3})/2.  Returns [nz, ny, nx, 3]
    (the z component is 0 in 2-D)."""
    out = torch.zeros(phi.shape + (3,), dtype=DTYPE)
    for a in range(model.lat.dim):
        d = AXIS_DIM[a]
        n = phi.shape[d]
        if model.walls[a]:
            g = torch.zeros_like(phi)
            idx = lambda i: torch.tensor([i])
            sel = lambda i: phi.index_select(d, idx(i))
            for i in range(n):
                if i == 0:
                    v = (-3.0 * sel(0) + 4.0 * sel(1) - sel(2)) / 2.0
                elif i == n - 1:
                    v = (3.0 * sel(n - 1) - 4.0 * sel(n - 2) + sel(n - 3)) / 2.0
                else:
                    v = (sel(i + 1) - sel(i - 1)) / 2.0
                g.index_copy_(d, idx(i), v)
        else:
            g = (torch.roll(phi, -1, dims=d) - torch.roll(phi, 1, dims=d)) / 2.0
        out[..., a] = g
    return out


def pressure_forcing(model, rho_i, u):
    """Pressure contribution of eq. (improved_forcing_scheme):
    S_p = omega [(e e - c_s^2 I)/c_s^4 . u] . grad(rho_i c_s^2)
        = omega [(e.u)(e.G) - c_s^2 u.G]/c_s^4,  G = c_s^2 grad rho_i
    (c_s of species i is constant); gradient of reading R6."""
    e = model.velocities()
    w = model.lat.w
    cs2l = model.sound2()
    G = torch.stack([cs2l[i] * gradient(model, rho_i[i]) for i in range(model.N)])
    cs2 = torch.tensor(cs2l, dtype=DTYPE)[:, None, None, None, None]
    eu = torch.einsum("nqc,zyxc->nqzyx", e, u)
    eG = torch.einsum("nqc,nzyxc->nqzyx", e, G)
    uG = _dot(u[None], G)[:, None]
    return w[None, :, None, None, None] * (eu * eG - cs2 * uG) / (cs2 * cs2)


def density_forcing(model, rho_i, rho, ueq):
    """Density contribution of eq. (improved_forcing_scheme):
    S_rho = omega [(e e - c_s^2 I)/c_s^2 . u_i^eq] . (w_i grad rho)
          = omega w_i [(e.u_i^eq)(e.grad rho) - c_s^2 u_i^eq.grad rho]/c_s^2,
    w_i = rho_i/rho the mass fraction; gradient of reading R6."""
    e = model.velocities()
    w = model.lat.w
    cs2 = torch.tensor(model.sound2(), dtype=DTYPE)[:, None, None, None, None]
    gr = gradient(model, rho)                               # [nz, ny, nx, 3]
    eu = torch.einsum("nqc,nzyxc->nqzyx", e, ueq)
    eg = torch.einsum("nqc,zyxc->nqzyx", e, gr)
    ug = _dot(ueq, gr[None])[:, None]
    wi = (rho_i / rho)[:, None]
    return w[None, :, None, None, None] * wi * (eu * eg - cs2 * ug) / cs2


def collide(model, f):
    """f~ = f + Omega^ii + sum_{j!=i} Omega^ij + (1 - dt/(2 tau_i)) S, with
    Omega^ii = -(f - f^(0))/tau_i                        (eq. BGK_self_collision)
    Omega^ij = -(1/tau_ij)(rho_j/rho) f^(eq)/c_s^2 (e-u).(u_i^eq - u_j^eq)
                                                   (eq. Cross_collision_Sirovich)
    inside eq. (LBE_forcing).  With model.forcing == "diff" the forcing term
    S includes the diffusion-driven contribution S_diff of eq.
    (improved_forcing_scheme); with "full" it is that whole equation,
    S - S_p + S_rho + S_diff."""
    N = model.N
    rho_i, ueq = species_moments(model, f)
    rho, u, n, p = mixture(model, rho_i, ueq)
    Y = cross_relaxation(model, rho_i, rho, n, p)
    feq, f0 = equilibria(model, rho_i, ueq, u)
    S = forcing_term(model, rho_i, u)
    if model.forcing in ("diff", "full"):
        S = S + diffusion_forcing(model, theta(model, rho_i, rho, ueq, Y), u)
    if model.forcing == "full":
        S = S - pressure_forcing(model, rho_i, u) + density_forcing(model, rho_i, rho, ueq)
    e = model.velocities()
    cs2 = model.sound2()
    tau = model.taus()
    out = []
    for i in range(N):
        omega_self = -(f[i] - f0[i]) / tau[i]
        e_minus_u = e[i][:, None, None, None, :] - u[None]          # [Q, z, y, x, 3]
        cross = torch.zeros_like(f[i])
        for j in range(N):
            if j == i:
                continue
            dv = ueq[i] - ueq[j]                                     # [z, y, x, 3]
            proj = _dot(e_minus_u, dv[None])
            cross = cross - Y[i, j][None] * (rho_i[j] / rho)[None] \
                * feq[i] / cs2[i] * proj
        out.append(f[i] + omega_self + cross + (1.0 - 0.5 / tau[i]) * S[i])
    return torch.stack(out)


# --------------------------------------------------------------------- stream
def _shift_source(model, plane, k):
    """Value of `plane` at O + k for every target O: periodic axes wrap, a
    source outside a wall axis is solid and contributes nothing."""
    out = plane
    for a in range(3):
        if k[a] == 0:
            continue
        dim = AXIS_DIM[a]
        out = torch.roll(out, shifts=-k[a], dims=dim)
        if model.walls[a]:
            n = model.shape_axis(a)
            idx = torch.arange(n)
            solid = (idx + k[a] < 0) | (idx + k[a] >= n)
            shape = [1, 1, 1]
            shape[dim] = n
            out = out * (~solid).to(DTYPE).reshape(shape)
    return out


def _wall_returns(model, ft, lam, walled):
    """The impermeable-wall terms of Appendix A (readings R2, R11), read as
    the return of what a wall-layer population would stream beyond the walls:
    source f~_beta(O) at a node O next to walls sends weight Lambda_k(e_beta)
    to the target O - k; for each set R of walls that such targets lie beyond,
    the lost weight
        prod_{a in R} lambda_{-s_a}(e_beta,a) prod_{a next to O, not in R}
        (1 - lambda_{-s_a}(e_beta,a))
    (s_a = -1 at the low wall of axis a, +1 at the high one) is returned to O,
    into the reversed direction if beta moves toward a wall of R, else into
    beta itself.  With one wall this is term by term the Appendix A rule
    (lambda_{-s}(e_alpha) f~_alpha(O) + lambda_{-s}(e_alphabar) f~_alphabar(O)
    for alpha pointing away from the wall); at c = 1 it is halfway
    bounce-back, also into corners; every source keeps its whole weight, so
    species mass is conserved."""
    N, Q = model.N, model.lat.Q
    dirs, opp = model.lat.dirs, model.lat.opp
    add = torch.zeros_like(ft)
    choices = []
    for a in walled:
        n = model.shape_axis(a)
        choices.append([(-1, 0), (1, n - 1)] + ([(0, None)] if n > 2 else []))
    import itertools
    for pat in itertools.product(*choices):
        adj = [(a, s) for a, (s, _) in zip(walled, pat) if s != 0]
        if not adj:
            continue
        # nodes of this adjacency pattern
        mask = torch.ones(model.nz, model.ny, model.nx, dtype=torch.bool)
        for a, (s, idx) in zip(walled, pat):
            d = AXIS_DIM[a] + 4                               # spatial dim in [nz, ny, nx]
            n = model.shape_axis(a)
            sel = torch.zeros(n, dtype=torch.bool)
            if s == 0:
                sel[1:n - 1] = True
            else:
                sel[idx] = True
            shape = [1, 1, 1]
            shape[d - 1] = n
            mask = mask & sel.reshape(shape)
        C = torch.zeros(N, Q, Q, dtype=DTYPE)                # [species, dest, source]
        for r in range(1, len(adj) + 1):
            for R in itertools.combinations(range(len(adj)), r):
                for i in range(N):
                    for b in range(Q):
                        lost = 1.0
                        toward = False
                        for t, (a, s) in enumerate(adj):
                            lm = lam[i][b][a][-s + 1]
                            if t in R:
                                lost *= lm
                                toward = toward or s * dirs[b][a] > 0
                            else:
                                lost *= 1.0 - lm
                        if lost != 0.0:
                            C[i, opp[b] if toward else b, b] += lost
        ret = torch.einsum("ndb,nbzyx->ndzyx", C, ft)
        add = add + torch.where(mask[None, None], ret, torch.zeros_like(ret))
    return add


def stream(model, ft):
    """Pull streaming with the second-order interpolation of eq.
    (Second_order_spatial_interpolation) (reading R1), generalised to
    3-D as the product of the 1-D factors, followed by the impermeable-wall
    scheme of Appendix A (reading R2).

    f^i_alpha(O) = sum_k prod_a lambda_{k_a}(e^i_{alpha,a}) f~^i_alpha(O + k)
    over k in {-1,0,1}^d with O + k a fluid node.  Species 1 (c = 1) reduces to
    the exact shift f(O) = f~(O - e).

    Wall scheme (Appendix A, the equations for right, left, upper and bottom
    walls): at a node O next to a wall on the side sigma (= +1 for the wall at
    the high end of axis a, -1 for the low end), for every alpha pointing away
    from that wall (sigma * c_alpha,a < 0) add the parts of f~_alpha(O) and
    f~_alphabar(O) that would have been streamed into the solid layer:
        + lambda_{-sigma}(e_alpha,a) f~_alpha(O)
        + lambda_{-sigma}(e_alphabar,a) f~_alphabar(O).
    """
    N, Q = model.N, model.lat.Q
    e = model.velocities()
    dim = model.lat.dim
    offs = [(kx, ky, kz) for kz in ((-1, 0, 1) if dim == 3 else (0,))
            for ky in (-1, 0, 1) for kx in (-1, 0, 1)]
    # Lambda_k(e^i_alpha) for every species, direction and source offset.
    lam = [[[lagrange_weights(float(e[i, al, a])) for a in range(3)]
            for al in range(Q)] for i in range(N)]
    out = torch.zeros_like(ft)
    for k in offs:
        wk = torch.tensor([[lam[i][al][0][k[0] + 1] * lam[i][al][1][k[1] + 1]
                            * lam[i][al][2][k[2] + 1] for al in range(Q)]
                           for i in range(N)], dtype=DTYPE)
        if not bool((wk != 0).any()):
            continue
        out = out + wk[:, :, None, None, None] * _shift_source(model, ft, k)
    # Appendix A wall terms (reading R2; reading R11 where walls meet).
    walled = [a for a in range(3) if model.walls[a]]
    if walled:
        out = out + _wall_returns(model, ft, lam, walled)
    if model.wall_velocity is not None:
        out = moving_wall_terms(model, out)
    return out


def moving_wall_terms(model, f):
    """Moving-wall term of Appendix A (the closing remark on non-stationary
    walls): at a node O next to a wall moving with tangential velocity u_w,
    every direction alpha pointing away from the wall gains
        + 2 omega_alpha rho_i w_i (e^i_alpha . u_w) / c_{s,i}^2,
    the paper's -2 omega rho_i w_i (e_alphabar . u_w)/c_s^2 written for the
    reflected direction (e_alpha = -e_alphabar).  Reading R10: rho_i and the
    mass fraction w_i = rho_i/rho are those of the streamed populations at O
    (the term adds no mass, so they are the same before and after it).
    f: streamed populations after the Appendix A terms."""
    N, Q = model.N, model.lat.Q
    e = model.velocities()                                  # [N, Q, 3]
    cs2 = model.sound2()
    a = [ax for ax in range(3) if model.walls[ax]][0]
    d = AXIS_DIM[a]
    n = model.shape_axis(a)
    out = f.clone()
    for side, layer in ((0, 0), (1, n - 1)):
        uw = model.wall_velocity[side]
        if not bool((uw != 0).any()):
            continue
        sigma = -1 if side == 0 else 1
        here = f.select(d, layer)                            # [N, Q, ., .]
        rho_i = here.sum(dim=1)                              # [N, ., .]
        w_i = rho_i / rho_i.sum(dim=0, keepdim=True)
        add = torch.zeros_like(here)
        for i in range(N):
            for al in range(Q):
                if sigma * model.lat.dirs[al][a] >= 0:
                    continue
                eu = float(e[i, al] @ uw)
                add[i, al] = 2.0 * float(model.lat.w[al]) * rho_i[i] * w_i[i] * eu / cs2[i]
        idx = [slice(None)] * 5
        idx[d] = layer
        out[tuple(idx)] = out[tuple(idx)] + add
    return out


def stream_equilibrium_walls(model, ft):
    """The comparison boundary of Sec. 4.1 (the equilibrium scheme set against
    the proposed wall scheme for the Ga = 0 Loschmidt tube): the solid nodes
    beyond a wall hold f = f^(0)(rho_s, u = 0) = w_alpha rho_s, with rho_s the
    density of the adjacent fluid node (the wall-layer node at the same
    tangential position), and the fluid streams from them with the same
    interpolation as from any node; no Appendix A terms.  A negative control:
    the paper shows that it does not conserve mass."""
    N, Q = model.N, model.lat.Q
    e = model.velocities()
    dim = model.lat.dim
    rho = ft.sum(dim=1)                                     # [N, nz, ny, nx]
    w = model.lat.w
    offs = [(kx, ky, kz) for kz in ((-1, 0, 1) if dim == 3 else (0,))
            for ky in (-1, 0, 1) for kx in (-1, 0, 1)]
    lam = [[[lagrange_weights(float(e[i, al, a])) for a in range(3)]
            for al in range(Q)] for i in range(N)]
    out = torch.zeros_like(ft)
    for k in offs:
        wk = torch.tensor([[lam[i][al][0][k[0] + 1] * lam[i][al][1][k[1] + 1]
                            * lam[i][al][2][k[2] + 1] for al in range(Q)]
                           for i in range(N)], dtype=DTYPE)
        if not bool((wk != 0).any()):
            continue
        fluid = _shift_source(model, ft, k)                 # 0 at solid sources
        # rho_s of the adjacent fluid node: clamp the source into the lattice
        # along the wall axis, shift as usual along the others
        rs = rho
        solid = torch.zeros(rho.shape[1:], dtype=torch.bool)
        for a in range(3):
            if k[a] == 0:
                continue
            d = AXIS_DIM[a]
            n = model.shape_axis(a)
            if model.walls[a]:
                idx = torch.clamp(torch.arange(n) + k[a], 0, n - 1)
                rs = rs.index_select(d, idx)
                bad = (torch.arange(n) + k[a] < 0) | (torch.arange(n) + k[a] >= n)
                shape = [1, 1, 1]
                shape[d] = n
                solid = solid | bad.reshape(shape)
            else:
                rs = torch.roll(rs, shifts=-k[a], dims=d)
        eq = w[None, :, None, None, None] * rs[:, None] * solid.to(DTYPE)[None, None]
        out = out + wk[:, :, None, None, None] * (fluid + eq)
    return out


def step(model, f):
    """One time step: f(t) -> f(t+1) = stream(collide(f(t)))."""
    return stream(model, collide(model, f))


def run(model, f, steps):
    for _ in range(steps):
        f = step(model, f)
    return f


# ----------------------------------------------------------------------- init
def initial_populations(model, x0):
    """Initial state from mole fractions x0 [N, nz, ny, nx].

    rho_i = x_i M_i n (Sec. 4.1) with n from default_n0; zero species and
    mixture velocity; the force-consistent initial velocity
    u_i0 = u_i^eq - F_i dt/(2 rho_i) = -k/2 replaces u_i^eq in eq. (feqi0)
    (Sec. 4.2), so with u = 0:  f = [1 + e.u_i0/c_s^2] omega rho_i."""
    x0 = torch.as_tensor(x0, dtype=DTYPE)
    M = torch.tensor(model.M, dtype=DTYPE)
    n = model.default_n0()
    rho_i = x0 * M[:, None, None, None] * n
    e = model.velocities()
    w = model.lat.w
    cs2 = torch.tensor(model.sound2(), dtype=DTYPE)[:, None, None, None, None]
    k = model.accel().permute(1, 2, 3, 0)                   # [nz, ny, nx, 3]
    ui0 = -0.5 * k
    e_u = torch.einsum("nqc,zyxc->nqzyx", e, ui0)
    return (1.0 + e_u / cs2) * w[None, :, None, None, None] * rho_i[:, None]


# ---------------------------------------------------------------- observables
def observables(model, f):
    """Macroscopic fields of a post-stream state f(t) (Sec. 2: moments are
    taken once streaming and boundary conditions are done):
      x_i = rho_i / (M_i n)                         (Sec. 3, x_i = rho_i/(n M_i))
      Theta_i = sum_j rho_i rho_j/(rho tau_ij) (u_i^eq - u_j^eq)
                                                   (eq. CE_theta_definition)
      u_i = u_i^eq - dt Theta_i/(2 rho_i)            (eq. CE_EQ83)
    (Theta_i/rho_i by theta_per_density, so a species with rho_i = 0 takes the
    limit, reading R12), plus rho_i, u_i^eq, rho, u, n, p and the FP64 total
    mass of each species."""
    rho_i, ueq = species_moments(model, f)
    rho, u, n, p = mixture(model, rho_i, ueq)
    Y = cross_relaxation(model, rho_i, rho, n, p)
    M = torch.tensor(model.M, dtype=DTYPE)
    x = rho_i / (M[:, None, None, None] * n)
    th = theta(model, rho_i, rho, ueq, Y)
    u_real = ueq - 0.5 * theta_per_density(model, rho_i, rho, ueq, Y)
    return {
        "rho_i": rho_i, "ueq": ueq, "rho": rho, "u": u, "n": n, "p": p,
        "x": x, "tau_inv": Y, "theta": th, "u_i": u_real,
        "mass": rho_i.sum(dim=(1, 2, 3)),
    }
