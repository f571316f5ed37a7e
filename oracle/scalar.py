"""A second, independent implementation of one time step, node by node in
plain Python floats.  It exists only to cross-check ``oracle.evd`` by brute
force on tiny lattices, so it is deliberately written differently:

* the cross-relaxation times solve eq. (relation_tauij_diff_coeff) for all
  pairs at once, as one P x P system (P = N(N-1)/2) eliminated by hand with
  partial pivoting, instead of column by column;
* the forcing term uses the expanded scalar form
  S = omega [ (e-u).F / c^2 + (e.u)(e.F) / c^4 ], which equals eq.
  (CE_forcing_term_discretized) term by term;
* streaming is done in PUSH form: each post-collision population is scattered
  to the targets that eq. (Second_order_spatial_interpolation) feeds from it,
  and every share whose target is a solid node is handed back, at the source
  node, to whichever of alpha / alphabar points away from that wall -- which is
  how Appendix A motivates its scheme (the terms that would have gone into the
  solid node A become contributions to f_alphabar(O) and f_alpha(O)).

Arrays are nested Python lists indexed [species][direction][z][y][x].
"""
import math

from .lattice import D2Q9_DIRS, D2Q9_W, D3Q19_DIRS, D3Q19_W


class ScalarModel:
    def __init__(self, lattice, nx, ny, nz, masses, diff, tau1, g, walls, n0=None):
        if lattice == "D2Q9":
            self.dirs, self.w = D2Q9_DIRS, [float(x) for x in D2Q9_W]
        else:
            self.dirs, self.w = D3Q19_DIRS, [float(x) for x in D3Q19_W]
        self.dim = 2 if lattice == "D2Q9" else 3
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = len(masses)
        self.M = [m / masses[0] for m in masses]
        self.D = [[float(diff[i][j]) for j in range(self.N)] for i in range(self.N)]
        self.tau1 = tau1
        self.g = [float(v) for v in g]
        self.walls = list(walls)
        self.c = [math.sqrt(1.0 / m) for m in self.M]
        self.cs2 = [c * c / 3.0 for c in self.c]
        self.tau = [0.5 + (tau1 - 0.5) * m for m in self.M]
        self.n0 = (1.0 / max(self.M)) if n0 is None else n0
        Q = len(self.dirs)
        self.opp = []
        for a in range(Q):
            d = self.dirs[a]
            self.opp.append(self.dirs.index((-d[0], -d[1], -d[2])))

    def size(self, axis):
        return (self.nx, self.ny, self.nz)[axis]

    # ------------------------------------------------------------- tau solve
    def pair_inverse_taus(self, rho_i):
        """All y_ij = 1/tau_ij of one node from one P x P linear system."""
        N, M, D = self.N, self.M, self.D
        rho = sum(rho_i)
        n = sum(rho_i[s] / M[s] for s in range(N))
        p = n * M[0] * self.cs2[0]
        pairs = [(i, j) for j in range(N) for i in range(j)]
        col = {pq: k for k, pq in enumerate(pairs)}

        def var(a, b):
            return col[(min(a, b), max(a, b))]

        P = len(pairs)
        A = [[0.0] * P for _ in range(P)]
        b = [0.0] * P
        for r, (i, j) in enumerate(pairs):
            Dij = D[i][j]
            A[r][r] += (rho_i[i] + rho_i[j]) / Dij + 2.0 * n * n * M[i] * M[j] / p
            for s in range(N):
                if s != i and s != j:
                    A[r][var(s, j)] += rho_i[s] / Dij
            b[r] = 2.0 * rho / Dij
        # Gaussian elimination with partial pivoting.
        for k in range(P):
            piv = max(range(k, P), key=lambda r: abs(A[r][k]))
            A[k], A[piv] = A[piv], A[k]
            b[k], b[piv] = b[piv], b[k]
            for r in range(k + 1, P):
                fac = A[r][k] / A[k][k]
                for cidx in range(k, P):
                    A[r][cidx] -= fac * A[k][cidx]
                b[r] -= fac * b[k]
        y = [0.0] * P
        for k in range(P - 1, -1, -1):
            acc = b[k] - sum(A[k][cidx] * y[cidx] for cidx in range(k + 1, P))
            y[k] = acc / A[k][k]
        Y = [[0.0] * N for _ in range(N)]
        for (i, j), k in col.items():
            Y[i][j] = Y[j][i] = y[k]
        return Y

    # --------------------------------------------------------------- collide
    def collide_node(self, fn):
        """fn[i][a] -> post-collision values for one node."""
        N, Q = self.N, len(self.dirs)
        g = self.g
        rho_i, ueq = [], []
        for i in range(N):
            r = sum(fn[i])
            m = [sum(self.c[i] * self.dirs[a][d] * fn[i][a] for a in range(Q))
                 for d in range(3)]
            rho_i.append(r)
            if r == 0.0:
                ueq.append([0.5 * g[d] for d in range(3)])
            else:
                ueq.append([m[d] / r + 0.5 * g[d] for d in range(3)])
        rho = sum(rho_i)
        u = [sum(rho_i[i] * ueq[i][d] for i in range(N)) / rho for d in range(3)]
        Y = self.pair_inverse_taus(rho_i)
        uu = sum(v * v for v in u)
        out = []
        for i in range(N):
            c2 = self.cs2[i]
            F = [rho_i[i] * g[d] for d in range(3)]
            row = []
            for a in range(Q):
                e = [self.c[i] * self.dirs[a][d] for d in range(3)]
                eu = sum(e[d] * u[d] for d in range(3))
                feq = self.w[a] * rho_i[i] * (1.0 + eu / c2 + eu * eu / (2 * c2 * c2)
                                              - uu / (2 * c2))
                emu = [e[d] - u[d] for d in range(3)]
                f0 = feq * (1.0 + sum(emu[d] * (ueq[i][d] - u[d]) for d in range(3)) / c2)
                cross = 0.0
                for j in range(N):
                    if j != i:
                        proj = sum(emu[d] * (ueq[i][d] - ueq[j][d]) for d in range(3))
                        cross -= Y[i][j] * (rho_i[j] / rho) * feq / c2 * proj
                eF = sum(e[d] * F[d] for d in range(3))
                S = self.w[a] * (sum(emu[d] * F[d] for d in range(3)) / c2
                                 + eu * eF / (c2 * c2))
                row.append(fn[i][a] - (fn[i][a] - f0) / self.tau[i] + cross
                           + (1.0 - 0.5 / self.tau[i]) * S)
            out.append(row)
        return out

    # ---------------------------------------------------------------- stream
    @staticmethod
    def _lam(s):
        return {-1: s * (1 + s) / 2, 0: 1 - s * s, 1: -s * (1 - s) / 2}

    def push_stream(self, ft):
        N, Q = self.N, len(self.dirs)
        nx, ny, nz = self.nx, self.ny, self.nz
        out = [[[[[0.0] * nx for _ in range(ny)] for _ in range(nz)]
                for _ in range(Q)] for _ in range(N)]
        ks = [-1, 0, 1]
        kz_list = ks if self.dim == 3 else [0]
        for i in range(N):
            for a in range(Q):
                e = [self.c[i] * self.dirs[a][d] for d in range(3)]
                lx, ly, lz = self._lam(e[0]), self._lam(e[1]), self._lam(e[2])
                for z in range(nz):
                    for y in range(ny):
                        for x in range(nx):
                            val = ft[i][a][z][y][x]
                            for kz in kz_list:
                                for ky in ks:
                                    for kx in ks:
                                        wgt = lx[kx] * ly[ky] * lz[kz]
                                        if wgt == 0.0:
                                            continue
                                        # this source feeds the target T = X - k
                                        T = [x - kx, y - ky, z - kz]
                                        hit = None
                                        for ax in range(3):
                                            nax = self.size(ax)
                                            if self.walls[ax]:
                                                if T[ax] < 0:
                                                    hit = (ax, -1)
                                                elif T[ax] >= nax:
                                                    hit = (ax, +1)
                                            else:
                                                T[ax] %= nax
                                        if hit is None:
                                            out[i][a][T[2]][T[1]][T[0]] += wgt * val
                                        else:
                                            ax, sigma = hit
                                            # hand back to the direction that points
                                            # away from the wall that was hit
                                            if sigma * self.dirs[a][ax] < 0:
                                                beta = a
                                            else:
                                                beta = self.opp[a]
                                            out[i][beta][z][y][x] += wgt * val
        return out

    def step(self, f):
        N, Q = self.N, len(self.dirs)
        ft = [[[[[0.0] * self.nx for _ in range(self.ny)] for _ in range(self.nz)]
               for _ in range(Q)] for _ in range(N)]
        for z in range(self.nz):
            for y in range(self.ny):
                for x in range(self.nx):
                    fn = [[f[i][a][z][y][x] for a in range(Q)] for i in range(N)]
                    post = self.collide_node(fn)
                    for i in range(N):
                        for a in range(Q):
                            ft[i][a][z][y][x] = post[i][a]
        return self.push_stream(ft)
