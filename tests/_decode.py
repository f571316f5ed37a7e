"""Test-side decoding of the library's stored state (the storage form the C
ABI documents: plane 0 of a species holds P0 = f~_0, plane a >= 1 holds
g_a = f~_a - (w_a/w_0) P0), written here so that the tests do not depend on
any decoding in the package."""
import torch

WEIGHTS = {9: [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
           19: [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12}


def decode(raw):
    """Post-collision populations f~ [N, Q, ...] in float64 from a stored state
    [N, Q, ...]: f~_0 = P0 and f~_a = (w_a/w_0) P0 + g_a."""
    r = raw.double()
    Q = r.shape[1]
    w = torch.tensor(WEIGHTS[Q], dtype=torch.float64, device=r.device)
    shape = (1, Q) + (1,) * (r.dim() - 2)
    f = (w / w[0]).view(shape) * r[:, :1] + r
    f[:, 0] = r[:, 0]
    return f


def encode(f):
    """The stored state [N, Q, ...] of populations f~ (float64), the inverse of
    decode (before rounding to float32)."""
    Q = f.shape[1]
    w = torch.tensor(WEIGHTS[Q], dtype=torch.float64, device=f.device)
    shape = (1, Q) + (1,) * (f.dim() - 2)
    s = f - (w / w[0]).view(shape) * f[:, :1]
    s[:, 0] = f[:, 0]
    return s


def populations(sim, which="cur", lattice=0):
    """f~ [N, Q, nz, ny, nx] (float64) of one lattice of a context."""
    return decode(sim.raw(which, lattice))


def densities(state):
    """rho_i = P0/w_0 + sum_{a>=1} g_a of a stored state [N, Q, ...] (float64)."""
    s = state.double()
    return s[:, 0] / WEIGHTS[s.shape[1]][0] + s[:, 1:].sum(dim=1)


def mole_fractions(state, masses):
    """x_i = rho_i/(M_i n), n = sum_j rho_j/M_j, of a stored state."""
    rho = densities(state)
    M = torch.tensor([m / masses[0] for m in masses], dtype=torch.float64,
                     device=rho.device).view(-1, *([1] * (rho.dim() - 1)))
    nm = rho / M
    return nm / nm.sum(dim=0, keepdim=True)
