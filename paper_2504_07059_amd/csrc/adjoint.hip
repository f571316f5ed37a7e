// Discrete adjoint of the fused step (reverse mode, written by hand).
//
// The forward step maps the stored state s(t-1) to s(t) = T C(S(T^-1 s(t-1))),
// with S the pull streaming with walls, C the collision, and T the linear
// change of variables of the storage (P0 = f~_0, g_a = f~_a - (w_a/w_0) f~_0).
// One reverse step, given lam_s(t) = dL/ds(t) and s(t-1):
//   kernel A (per node): f(t) = S(T^-1 s(t-1)) by the forward gather;
//            lam_f = T^T lam_s(t); mu = (dC/df)^T lam_f at f(t), stored in a
//            scratch buffer (population space); parameter gradients
//            (dC/dD)^T lam_f and (dC/dg)^T lam_f accumulated in FP64;
//   kernel B (per node): lam_f(t-1) = S^T mu, i.e. the gather of mu with the
//            velocities reversed plus the transposed wall terms; stored as
//            lam_s(t-1) = T^-T lam_f(t-1).
// Both kernels run one wave per species over tiles of 64 columns (their own
// tile list, independent of the forward step's execution shape).  The state
// and adjoint are FP32; parameter gradients are summed in FP64 per thread,
// per work-group and then over work-groups in a fixed order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "adjoint.hpp"
#include "kernels.hpp"

namespace lbmmc {

// Block reduction of NG doubles, ADDED into this work-group's own partials
// (each slot has one writer, and the reverse steps of a sequence run in
// stream order, so the per-tile sums accumulate deterministically).
template <int NG>
__device__ __forceinline__ void block_reduce_add(double (&acc)[NG], double* __restrict__ out) {
    __shared__ double red[4][NG];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wave = tid >> 6;
    const int nwaves = (blockDim.x * blockDim.y + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (tid < NG) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[w][tid];
        out[tid] += s;
    }
}

// ------------------------------------------------------------------ kernel A
// One wave per species over 64 columns.  Per layer: the wave gathers f(t) of
// its species from f~(t-1) and publishes its density and momentum in LDS;
// every wave recomputes the node's forward collision state; each wave runs
// its species' part of the reverse sweep and publishes its contributions to
// the shared adjoints (u, rho, the densities and velocities, y); every wave
// sums them in species order and runs the shared tail (mixture and
// cross-relaxation reverse), then finishes and stores its own species' mu.
template <int LAT, int NS, int POL>
struct AdjSplitOp {
    static constexpr int Q = Lat<LAT>::Q;
    static constexpr int NG = NS * (NS - 1) / 2 + 3;
    static constexpr int KX = 4 + 5 * NS;   // packed contribution floats per species
    Buf lam;      // lam_s(t), representation space
    Buf mu;       // scratch, population space
    CollConst C;
    float (*x1)[4][64];
    float (*x2)[KX][64];
    int s, lane;
    bool inside;
    double acc[NG];
    __device__ __forceinline__ void operator()(float P0, float (&F)[Q], int, unsigned own) {
        using L = Lat<LAT>;
        // own density and momentum (sum_a w_a = 1, sum_a c_a w_a = 0)
        float sf = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            const float v = F[a];
            sf += v;
            jx += (float)L::cx(a) * v;
            jy += (float)L::cy(a) * v;
            jz += (float)L::cz(a) * v;
        }
        x1[s][0][lane] = fmaf(P0, L::inv_w0, sf);
        x1[s][1][lane] = jx;
        x1[s][2][lane] = jy;
        x1[s][3][lane] = jz;
        // lam_f = T^T lam_s: lam_f0 = lam_P0 - sum_a (w_a/w_0) lam_ga, lam_fa = lam_ga
        float lt[Q];
        float l0 = ldb(lam, s * Q, own);
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            lt[a] = ldb(lam, s * Q + a, own);
            l0 = fmaf(-L::wr(a), lt[a], l0);
        }
        lt[0] = l0;
        __syncthreads();
        float rho[NS], jm[NS][3];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            rho[j] = x1[j][0][lane];
            jm[j][0] = x1[j][1][lane];
            jm[j][1] = x1[j][2][lane];
            jm[j][2] = x1[j][3][lane];
        }
        VjpFwd<NS> f;
        vjp_forward<NS>(rho, jm, C, f);
        VjpAcc<NS> part;
        vjp_zero<NS>(part);
        float dg[3] = {0.0f, 0.0f, 0.0f};
        float row[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i != s) continue;
            vjp_species<LAT, NS>(i, rho, f, C, lt, part, dg);
#pragma unroll
            for (int j = 0; j < NS; ++j) row[j] = part.dY[i][j];
        }
        {
            int k = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) x2[s][k++][lane] = part.dU[d];
            x2[s][k++][lane] = part.dR;
#pragma unroll
            for (int j = 0; j < NS; ++j) x2[s][k++][lane] = part.drho[j];
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int d = 0; d < 3; ++d) x2[s][k++][lane] = part.due[j][d];
#pragma unroll
            for (int j = 0; j < NS; ++j) x2[s][k++][lane] = row[j];
        }
        __syncthreads();
        VjpAcc<NS> A;
        vjp_zero<NS>(A);
#pragma unroll
        for (int v = 0; v < NS; ++v) {
            int k = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) A.dU[d] += x2[v][k++][lane];
            A.dR += x2[v][k++][lane];
#pragma unroll
            for (int j = 0; j < NS; ++j) A.drho[j] += x2[v][k++][lane];
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int d = 0; d < 3; ++d) A.due[j][d] += x2[v][k++][lane];
#pragma unroll
            for (int j = 0; j < NS; ++j) A.dY[v][j] = x2[v][k++][lane];
        }
        float dK[NS][NS];
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = 0; j < NS; ++j) dK[i][j] = 0.0f;
        vjp_mixture<NS>(rho, f, C, A, dK);
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i != s) continue;
            vjp_finish<LAT, NS>(i, rho, f, C, A, lt, dg);
        }
        if (inside) {
#pragma unroll
            for (int a = 0; a < Q; ++a) stb<POL>(mu, s * Q + a, own, lt[a]);
            int k = 0;
            // every wave holds the same dL/dK: the species-0 wave adds it
#pragma unroll
            for (int i = 0; i < NS; ++i)
#pragma unroll
                for (int j = i + 1; j < NS; ++j) acc[k++] += s == 0 ? (double)dK[i][j] : 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) acc[k + d] += (double)dg[d];
        }
    }
};

template <int LAT, int NS, int POL>
__global__ void __launch_bounds__(256) k_adj_collide(const float* __restrict__ fprev,
                                                     const float* __restrict__ lam,
                                                     float* __restrict__ mu,
                                                     const LatParams* __restrict__ lps,
                                                     const Tile* __restrict__ tiles, int bx,
                                                     double* __restrict__ gpart) {
    constexpr int DIM = Lat<LAT>::DIM;
    constexpr int Q = Lat<LAT>::Q;
    using Op = AdjSplitOp<LAT, NS, POL>;
    __shared__ float x1[NS][4][64];
    __shared__ float x2[NS][Op::KX][64];
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const Tile T = tiles[blockIdx.x];
    const LatParams& P = lps[T.lat];
    int x, y;
    bool zero;
    const bool inside = tile_column<LAT>(T, P, lane, bx, x, y, zero);
    const int64_t lf = P.plane * NS * Q;
    Op op{make_buf(lam + P.base, lf, P.plane), make_buf(mu + P.base, lf, P.plane),
          coll_const(P), x1, x2, s, lane, inside, {}};
#pragma unroll
    for (int q = 0; q < Op::NG; ++q) op.acc[q] = 0.0;
    const GatherConst G = gather_const(P, DIM);
    const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
    march1<LAT>(make_buf(fprev + P.base, lf, P.plane), G, s, L, x, y, zero, bx == 64, T.m0,
                T.m1, op);
    block_reduce_add<Op::NG>(op.acc, gpart + (int64_t)blockIdx.x * Op::NG);
}

// ------------------------------------------------------------------ kernel B
// lam_f(t-1)(X) = sum_k Lambda_k(e) mu(X - k) over fluid targets (the gather
// with the velocity reversed: Lambda_{-k}(e) = Lambda_k(-e)), plus the
// transposed wall terms; species 1 (c = 1): mu_a(X + c_a), or mu_abar(X)
// where X + c_a is solid.  Stored as lam_s = T^-T lam_f:
// lam_P0 = lam_f0 + sum_a (w_a/w_0) lam_fa, lam_ga = lam_fa.  One thread per
// (column, species): species are independent here.
template <int LAT, int NS, int POL>
__global__ void __launch_bounds__(256) k_adj_stream(const float* __restrict__ mu,
                                                    float* __restrict__ lamout,
                                                    const LatParams* __restrict__ lps,
                                                    const Tile* __restrict__ tiles, int bx) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int DIM = La::DIM;
    constexpr int Q = La::Q;
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const Tile T = tiles[blockIdx.x];
    const LatParams& P = lps[T.lat];
    int x, y;
    bool zero;
    if (!tile_column<LAT>(T, P, lane, bx, x, y, zero)) return;
    const GatherConst G = gather_const(P, DIM);
    const int64_t lf = P.plane * NS * Q;
    const Buf M = make_buf(mu + P.base, lf, P.plane);
    const Buf O = make_buf(lamout + P.base, lf, P.plane);
    const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
    // (the reverse step is provided for at most one wall axis)
    const bool wx = (G.walls & 1) != 0, wy = DIM == 3 && (G.walls & 2) != 0,
               wm = (G.walls & (1 << Fr::MA)) != 0;
    const int xm = nbr(x, -1, G.nx, wx), xp = nbr(x, 1, G.nx, wx);
    int ym = 0, yp = 0;
    if (DIM == 3) {
        ym = nbr(y, -1, G.ny, wy);
        yp = nbr(y, 1, G.ny, wy);
    }
    const unsigned bxo[3] = {xm < 0 ? kSolid : (unsigned)(xm - x) * 4u, 0u,
                             xp < 0 ? kSolid : (unsigned)(xp - x) * 4u};
    const unsigned byo[3] = {DIM == 3 ? (ym < 0 ? kSolid : (unsigned)((ym - y) * G.pitch) * 4u) : 0u,
                             0u,
                             DIM == 3 ? (yp < 0 ? kSolid : (unsigned)((yp - y) * G.pitch) * 4u) : 0u};
    const int sx = wx ? (x == 0 ? -1 : (x == G.nx - 1 ? 1 : 0)) : 0;
    const int sy = wy ? (y == 0 ? -1 : (y == G.ny - 1 ? 1 : 0)) : 0;
    const unsigned colbase = (unsigned)((DIM == 2 ? 0 : y * G.pitch) + x) * 4u;
    const unsigned lsb = (unsigned)G.lstride * 4u;
    const int pb0 = s * Q;
    for (int m = T.m0; m < T.m1; ++m) {
        const int mmv = nbr(m, -1, G.nm, wm), mpv = nbr(m, 1, G.nm, wm);
        const unsigned own = (unsigned)m * lsb + colbase;
        const unsigned bmo[3] = {mmv < 0 ? kSolid : (unsigned)(mmv - m) * lsb, 0u,
                                 mpv < 0 ? kSolid : (unsigned)(mpv - m) * lsb};
        const int sm = wm ? (m == 0 ? -1 : (m == G.nm - 1 ? 1 : 0)) : 0;
        const int axis = wx ? 0 : (wm ? Fr::MA : 1);
        const int side = wx ? sx : (wm ? sm : sy);
        float lf_[Q];
        lf_[0] = ldb(M, pb0, own);
        if (s == 0) {
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                // reversed shift: mu_a(X + c_a), or the bounce-back transpose
                const int c0 = Fr::p0(a), c1 = Fr::p1(a), cm = Fr::pm(a);
                unsigned src = own;
                bool solid = false;
                if (c0 != 0) { src += bxo[1 + c0]; solid = solid || (c0 < 0 ? xm < 0 : xp < 0); }
                if (DIM == 3 && c1 != 0) { src += byo[1 + c1]; solid = solid || (c1 < 0 ? ym < 0 : yp < 0); }
                if (cm != 0) { src += bmo[1 + cm]; solid = solid || (cm < 0 ? mmv < 0 : mpv < 0); }
                const int lo = a < La::opp(a) ? a : La::opp(a);
                const unsigned sg = solid ? own + (unsigned)((La::opp(a) - lo) * M.pb)
                                          : src + (unsigned)((a - lo) * M.pb);
                lf_[a] = ldb(M, lo, sg);
            }
        } else {
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const int c0 = Fr::p0(a), c1 = Fr::p1(a), cm = Fr::pm(a);
                // weights of the reversed velocity: offsets k' with Lambda_k'(-e)
                const W3 wxw = wsel(-c0, L), wyw = wsel(-c1, L), wmw = wsel(-cm, L);
                const float wxv[3] = {wxw.m, wxw.z, wxw.p};
                const float wyv[3] = {wyw.m, wyw.z, wyw.p};
                const float wmv[3] = {wmw.m, wmw.z, wmw.p};
                float v = 0.0f;
#pragma unroll
                for (int km = -1; km <= 1; ++km) {
                    if (cm == 0 && km != 0) continue;
                    float vy = 0.0f;
#pragma unroll
                    for (int ky = -1; ky <= 1; ++ky) {
                        if ((DIM == 2 || c1 == 0) && ky != 0) continue;
                        float vx = 0.0f;
#pragma unroll
                        for (int kx = -1; kx <= 1; ++kx) {
                            if (c0 == 0 && kx != 0) continue;
                            const unsigned off = own + bmo[1 + km] + byo[1 + ky] + bxo[1 + kx];
                            vx = fmaf(wxv[1 + kx], ldb(M, pb0 + a, off), vx);
                        }
                        vy = fmaf(wyv[1 + ky], vx, vy);
                    }
                    v = fmaf(wmv[1 + km], vy, v);
                }
                // transposed walls
                if (side != 0) {
                    const int ca = Fr::comp(a, axis);
                    if (ca != 0) {
                        if (side * ca < 0) v = fmaf(L[2], ldb(M, pb0 + a, own), v);
                        else v = fmaf(L[0], ldb(M, pb0 + La::opp(a), own), v);
                    }
                }
                lf_[a] = v;
            }
        }
        float lp0 = lf_[0];
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            lp0 = fmaf(La::wr(a), lf_[a], lp0);
            stb<POL>(O, pb0 + a, own, lf_[a]);
        }
        stb<POL>(O, pb0, own, lp0);
    }
}

// ----------------------------------------------------------------- init VJP
// f~(0) = C(f(0; g)), f_ia(0) = w_a rho_i (1 - e.g/(2 c_s^2)): the collision
// VJP at f(0) plus df(0)/dg.
template <int LAT, int NS>
__global__ void __launch_bounds__(256) k_adj_init(const LatParams* __restrict__ lps,
                                                  const double* __restrict__ x0,
                                                  const float* __restrict__ lam,
                                                  double* __restrict__ gpart) {
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    constexpr int NG = NS * (NS - 1) / 2 + 3;
    const LatParams& P = lps[0];
    const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
    const CollConst C = coll_const(P);
    const Buf Lb = make_buf(lam + P.base, P.plane * NS * Q, P.plane);
    double acc[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) acc[q] = 0.0;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < nodes;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(id % P.nx);
        const int64_t r = id / P.nx;
        const int yy = (int)(r % P.ny);
        const int z = (int)(r / P.ny);
        const unsigned own = (unsigned)(((int64_t)z * P.ny + yy) * P.pitch + x) * 4u;
        float lt[NS][Q], rho[NS], jm[NS][3];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            rho[s] = (float)(x0[s * nodes + id] * (double)P.M[s] * (double)P.n0);
            const float c = C.c[s], ics = C.inv_cs2[s];
            jm[s][0] = jm[s][1] = jm[s][2] = 0.0f;
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const float eu = c * cdot<LAT>(a, -0.5f * C.g[0], -0.5f * C.g[1], -0.5f * C.g[2]);
                const float fa = L::w(a) * rho[s] * (1.0f + ics * eu);
                jm[s][0] += (float)L::cx(a) * fa;
                jm[s][1] += (float)L::cy(a) * fa;
                jm[s][2] += (float)L::cz(a) * fa;
            }
            float l0 = ldb(Lb, s * Q, own);
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                lt[s][a] = ldb(Lb, s * Q + a, own);
                l0 = fmaf(-L::wr(a), lt[s][a], l0);
            }
            lt[s][0] = l0;
        }
        float dK[NS][NS], dg[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = 0; j < NS; ++j) dK[i][j] = 0.0f;
        collide_vjp<LAT, NS>(rho, jm, lt, C, dK, dg);
        // f_ia(0) depends on g through -e.g/(2 c_s^2)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const float c = C.c[s], ics = C.inv_cs2[s];
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const float k = -0.5f * L::w(a) * rho[s] * ics * c * lt[s][a];
                dg[0] += k * L::cx(a);
                dg[1] += k * L::cy(a);
                dg[2] += k * L::cz(a);
            }
        }
        int k = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = i + 1; j < NS; ++j) acc[k++] += (double)dK[i][j];
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[k + d] += (double)dg[d];
    }
    block_reduce_add<NG>(acc, gpart + (int64_t)blockIdx.x * NG);
}

// Fixed-order sum of the per-block partials (one work-group of 256 threads:
// thread t takes blocks t, t+256, ...; then a fixed shuffle and LDS tree), with
// d/dK converted to d/dD (dK_ij/dD_ij = 6 M_i M_j), added into grad.
__global__ void __launch_bounds__(256) k_grad_reduce(const LatParams* __restrict__ lps,
                                                     const double* __restrict__ gpart,
                                                     int nblocks, int ng, int ns,
                                                     double* __restrict__ grad) {
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int npair = ns * (ns - 1) / 2;
    for (int q = 0; q < ng; ++q) {
        double v = 0.0;
        for (int b = tid; b < nblocks; b += 256) v += gpart[(int64_t)b * ng + q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (tid == 0) {
            double s = (red[0] + red[1]) + (red[2] + red[3]);
            if (q < npair) {
                int k = 0;
                for (int i = 0; i < ns; ++i)
                    for (int j = i + 1; j < ns; ++j, ++k)
                        if (k == q) s *= lps[0].dscale[i][j];
            }
            grad[q] += s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- launchers
template <int LAT, int NS>
static hipError_t adj_t(const Launch& L, const float* lam_in, float* mu, double* gpart) {
    if (L.bx * L.by != 64) return hipErrorInvalidValue;
    auto go = [&](auto pol) {
        hipLaunchKernelGGL((k_adj_collide<LAT, NS, decltype(pol)::value>), dim3(L.ntiles),
                           dim3(64, NS), 0, L.stream, L.src, lam_in, mu, L.lp, L.tiles, L.bx,
                           gpart);
    };
    if (L.wt)
        go(std::integral_constant<int, kStoreWT>{});
    else
        go(std::integral_constant<int, kStoreNT>{});
    return hipGetLastError();
}

hipError_t launch_adjoint(int lattice, int ns, const Launch& L, const float* lam_in, float* mu,
                          double* gpart, int) {
    if (lattice == 0) {
        if (ns == 2) return adj_t<0, 2>(L, lam_in, mu, gpart);
        if (ns == 3) return adj_t<0, 3>(L, lam_in, mu, gpart);
        if (ns == 4) return adj_t<0, 4>(L, lam_in, mu, gpart);
    } else {
        if (ns == 2) return adj_t<1, 2>(L, lam_in, mu, gpart);
        if (ns == 3) return adj_t<1, 3>(L, lam_in, mu, gpart);
        if (ns == 4) return adj_t<1, 4>(L, lam_in, mu, gpart);
    }
    return hipErrorInvalidValue;
}

template <int LAT, int NS>
static hipError_t adjs_t(const Launch& L, const float* mu, float* lam_out) {
    if (L.bx * L.by != 64) return hipErrorInvalidValue;
    auto go = [&](auto pol) {
        hipLaunchKernelGGL((k_adj_stream<LAT, NS, decltype(pol)::value>), dim3(L.ntiles),
                           dim3(64, NS), 0, L.stream, mu, lam_out, L.lp, L.tiles, L.bx);
    };
    if (L.wt)
        go(std::integral_constant<int, kStoreWT>{});
    else
        go(std::integral_constant<int, kStoreNT>{});
    return hipGetLastError();
}

hipError_t launch_adjoint_stream(int lattice, int ns, const Launch& L, const float* mu,
                                 float* lam_out) {
    if (lattice == 0) {
        if (ns == 2) return adjs_t<0, 2>(L, mu, lam_out);
        if (ns == 3) return adjs_t<0, 3>(L, mu, lam_out);
        if (ns == 4) return adjs_t<0, 4>(L, mu, lam_out);
    } else {
        if (ns == 2) return adjs_t<1, 2>(L, mu, lam_out);
        if (ns == 3) return adjs_t<1, 3>(L, mu, lam_out);
        if (ns == 4) return adjs_t<1, 4>(L, mu, lam_out);
    }
    return hipErrorInvalidValue;
}

template <int LAT, int NS>
static hipError_t adji_t(const LatParams* lp, const LatParams& h, const double* x0,
                         const float* lam0, double* gpart, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_init<LAT, NS>), dim3(nblocks), dim3(256), 0, s, lp, x0, lam0, gpart);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(int lattice, int ns, const LatParams* lp, const LatParams& h,
                               const double* x0, const float* lam0, double* gpart, int nblocks,
                               hipStream_t s) {
    if (lattice == 0) {
        if (ns == 2) return adji_t<0, 2>(lp, h, x0, lam0, gpart, nblocks, s);
        if (ns == 3) return adji_t<0, 3>(lp, h, x0, lam0, gpart, nblocks, s);
        if (ns == 4) return adji_t<0, 4>(lp, h, x0, lam0, gpart, nblocks, s);
    } else {
        if (ns == 2) return adji_t<1, 2>(lp, h, x0, lam0, gpart, nblocks, s);
        if (ns == 3) return adji_t<1, 3>(lp, h, x0, lam0, gpart, nblocks, s);
        if (ns == 4) return adji_t<1, 4>(lp, h, x0, lam0, gpart, nblocks, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_grad_reduce(const LatParams* lp, const double* gpart, int nblocks, int ng,
                              int ns, double* grad, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_reduce, dim3(1), dim3(256), 0, s, lp, gpart, nblocks, ng, ns, grad);
    return hipGetLastError();
}

}  // namespace lbmmc
