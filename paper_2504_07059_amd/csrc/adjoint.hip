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
// In a sequence of reverse steps, kernel B of one step and kernel A of the
// step before it run as one fused pass that gathers lam_f from the later
// step's mu directly (T^-T followed by T^T is the identity).
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
    Buf lam;      // lam_s(t), representation space (this species' view)
    Buf mu;       // scratch, population space (this species' view)
    CollConst C;
    float (*x1)[4][64];
    float (*x2)[KX][64];
    int s, lane;
    bool inside;
    // Build of the fused pass for three waves per SIMD: 2-D, up to three
    // species, states beyond the last-level cache (non-temporal stores).
    // Its marching and gradient sums then live in LDS and its stores are not
    // deferred; on cache-resident lattices, where one tile's chain sets the
    // step time, the register build is faster.
    static constexpr bool kThree = Lat<LAT>::DIM == 2 && NS <= 3 && POL == kStoreNT;
    // FP64 gradient sums of this lane: in registers, or in LDS (accl: this
    // lane's element of the wave's [NG][64] doubles) in 3-D, which keeps the
    // D3Q19 kernels at two waves per SIMD with four species, and for kThree
    static constexpr bool kLdsSums = Lat<LAT>::DIM == 3 || kThree;
    double accr[kLdsSums ? 1 : NG];
    double* accl;
    __device__ __forceinline__ double& acc(int q) {
        if constexpr (kLdsSums)
            return accl[q * 64];
        else
            return accr[q];
    }
    // 2-D, up to three species: the layer's mu is stored in the next layer's
    // call, after that layer's gathers have their loads back (with four
    // species the held values would cost the fused pass its second wave per
    // SIMD)
    static constexpr bool kDefer = Lat<LAT>::DIM == 2 && NS < 4 && !kThree;
    float out[Q];
    unsigned out_own;
    bool pend;
    __device__ __forceinline__ void flush() {
        if (pend) {
#pragma unroll
            for (int a = 0; a < Q; ++a) stb<POL>(mu, a, out_own, out[a]);
        }
        pend = false;
    }
    // kernel A alone: lam_f = T^T lam_s(t) from the stored adjoint
    __device__ __forceinline__ void operator()(float P0, float (&F)[Q], int, unsigned own) {
        using L = Lat<LAT>;
        // lam_f0 = lam_P0 - sum_a (w_a/w_0) lam_ga, lam_fa = lam_ga
        float lt[Q];
        float l0 = ldb(lam, 0, own);
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            lt[a] = ldb(lam, a, own);
            l0 = fmaf(-L::wr(a), lt[a], l0);
        }
        lt[0] = l0;
        reverse(P0, F, lt, own);
    }
    // fused reverse step: lam_f(t) given in population space (the transposed
    // stream of the later step's mu, computed by the caller)
    __device__ __forceinline__ void operator()(float P0, float (&F)[Q], float (&lt)[Q],
                                               unsigned own) {
        reverse(P0, F, lt, own);
    }
    // the collision VJP at f(t) = (P0, F) of lam_f = lt; lt becomes mu
    __device__ __forceinline__ void reverse(float P0, float (&F)[Q], float (&lt)[Q],
                                            unsigned own) {
        using L = Lat<LAT>;
        if constexpr (kDefer) flush();
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
            if constexpr (kDefer) {
#pragma unroll
                for (int a = 0; a < Q; ++a) out[a] = lt[a];
                out_own = own;
                pend = true;
            } else {
#pragma unroll
                for (int a = 0; a < Q; ++a) stb<POL>(mu, a, own, lt[a]);
            }
            int k = 0;
            // every wave holds the same dL/dK: the species-0 wave adds it
#pragma unroll
            for (int i = 0; i < NS; ++i)
#pragma unroll
                for (int j = i + 1; j < NS; ++j, ++k) acc(k) += s == 0 ? (double)dK[i][j] : 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) acc(k + d) += (double)dg[d];
        }
    }
    // the wave's sums, for the block reduction
    __device__ __forceinline__ void sums(double (&out)[NG]) {
#pragma unroll
        for (int q = 0; q < NG; ++q) out[q] = acc(q);
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
    using Op = AdjSplitOp<LAT, NS, POL>;
    __shared__ float x1[NS][4][64];
    __shared__ float x2[NS][Op::KX][64];
    __shared__ double gsum[Op::kLdsSums ? NS : 1][Op::NG][64];
    // 3-D: the march's partial sums of every wave
    __shared__ float msum[Lat<LAT>::DIM == 3 ? NS - 1 : 1][2 * kMarDirs<LAT>][64];
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const Tile T = tiles[blockIdx.x];
    const LatParams& P = lps[T.lat];
    int x, y;
    bool zero;
    const bool inside = tile_column<LAT>(T, P, lane, bx, x, y, zero);
    Op op{species_buf<LAT>(lam + P.base, P.plane, s), species_buf<LAT>(mu + P.base, P.plane, s),
          coll_const(P), x1, x2, s, lane, inside, {}, &gsum[Op::kLdsSums ? s : 0][0][lane]};
#pragma unroll
    for (int q = 0; q < Op::NG; ++q) op.acc(q) = 0.0;
    op.pend = false;
    const GatherConst G = gather_const(P, DIM);
    const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
    march1<LAT, Op, Lat<LAT>::DIM == 3>(species_buf<LAT>(fprev + P.base, P.plane, s), G, s, L, x,
                                         y, zero, bx == 64, T.m0, T.m1, op,
                                         &msum[Lat<LAT>::DIM == 3 && s > 0 ? s - 1 : 0][0][lane]);
    op.flush();
    double sums[Op::NG];
    op.sums(sums);
    block_reduce_add<Op::NG>(sums, gpart + (int64_t)blockIdx.x * Op::NG);
}

// ------------------------------------------------------------------ kernel B
// lam_f(t-1)(X) = sum_k Lambda_k(-e) mu(X + k) over fluid sources X + k (the
// pull gather with the velocity reversed: Lambda_{-k}(e) = Lambda_k(-e)),
// plus the transposed wall terms; species 1 (c = 1): mu_a(X + c_a), or
// mu_abar(X) where X + c_a is solid.  Stored as lam_s = T^-T lam_f:
// lam_P0 = lam_f0 + sum_a (w_a/w_0) lam_fa, lam_ga = lam_fa.
// The same march as the forward gather: one wave per species over a tile's
// columns, the cross-section passes read per layer (x neighbours across lanes
// for 64-column rows), the pass along the marching axis carried in registers
// (two partial sums per plane), so every value of mu is read about once.
// Direction a reversed has the components of opp(a).
#define LBM_HPR(CEN)                                                                      \
    ((Fr::p0(La::opp(a)) > 0)                                                             \
         ? ((Fr::p1(La::opp(a)) > 0)   ? hpass<LAT, 1, 1>(M, pidx, CEN, col, L, nb)        \
            : (Fr::p1(La::opp(a)) < 0) ? hpass<LAT, 1, -1>(M, pidx, CEN, col, L, nb)       \
                                       : hpass<LAT, 1, 0>(M, pidx, CEN, col, L, nb))       \
     : (Fr::p0(La::opp(a)) < 0)                                                           \
         ? ((Fr::p1(La::opp(a)) > 0)   ? hpass<LAT, -1, 1>(M, pidx, CEN, col, L, nb)       \
            : (Fr::p1(La::opp(a)) < 0) ? hpass<LAT, -1, -1>(M, pidx, CEN, col, L, nb)      \
                                       : hpass<LAT, -1, 0>(M, pidx, CEN, col, L, nb))      \
         : ((Fr::p1(La::opp(a)) > 0)   ? hpass<LAT, 0, 1>(M, pidx, CEN, col, L, nb)        \
            : (Fr::p1(La::opp(a)) < 0) ? hpass<LAT, 0, -1>(M, pidx, CEN, col, L, nb)       \
                                       : hpass<LAT, 0, 0>(M, pidx, CEN, col, L, nb)))

// Marching state of the reversed gather of one heavier species: the
// marching-axis partial sums of its planes of mu.
template <int LAT, bool LDS = false>
using RevMarch = MarchSums<LAT, LDS>;

// Start the reversed gather of species s (M: its view of mu) at layer m0.
template <int LAT, class NB, bool RL>
__device__ __forceinline__ void rev_begin(const Buf& M, const GatherConst& G, const ColGeom& g,
                                          int s, const float (&L)[3], int m0, RevMarch<LAT, RL>& r,
                                          const NB& nb) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    const Col& col = g.col;
    if (s == 0) return;
    const unsigned cm_ = layer_off(g, nbr(m0, -1, G.nm, g.wm)), c0_ = layer_off(g, m0);
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        if (Fr::pm(a) != 0) {
            const int pidx = a;
            const W3 wmar = wsel(-Fr::pm(a), L);
            const float hm = LBM_HPR(cm_);
            const float h0 = LBM_HPR(c0_);
            r.set(0, a, fmaf(wmar.z, h0, wmar.m * hm));
            r.set(1, a, wmar.m * h0);
        } else if constexpr (!RL) {
            r.set(0, a, 0.0f);
            r.set(1, a, 0.0f);
        }
    }
}

// lam_f(t-1) at layer m of the column (population space): the reversed
// gather of mu plus the transposed wall terms.
template <int LAT, class NB, bool RL>
__device__ __forceinline__ void rev_layer(const Buf& M, const GatherConst& G, const ColGeom& g,
                                          int s, const float (&L)[3], int m, unsigned own,
                                          unsigned nxt, RevMarch<LAT, RL>& r,
                                          float (&lf)[Lat<LAT>::Q], const NB& nb) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    constexpr int DIM = La::DIM;
    const Col& col = g.col;
    lf[0] = ldb(M, 0, own);
    if (s == 0) {
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            // source X + c_a (the reversed shift); where it is solid, the
            // bounce-back transpose mu_abar(X)
            const int c0 = Fr::p0(a), c1 = Fr::p1(a), cm = Fr::pm(a);
            unsigned src = own;
            bool solid = false;
            if (c0 > 0) { src += col.bxp; solid = solid || col.sxp; }
            if (c0 < 0) { src += col.bxm; solid = solid || col.sxm; }
            if constexpr (DIM == 3) {
                if (c1 > 0) { src += col.byp; solid = solid || col.syp; }
                if (c1 < 0) { src += col.bym; solid = solid || col.sym; }
            }
            if (cm != 0) {
                const int ms = nbr(m, cm, G.nm, g.wm);
                solid = solid || ms < 0;
                src += (unsigned)(ms - m) * g.lsb;
            }
            const int lo = a < La::opp(a) ? a : La::opp(a);
            const unsigned sg = solid ? own + (unsigned)((La::opp(a) - lo) * M.pb)
                                      : src + (unsigned)((a - lo) * M.pb);
            lf[a] = ldb(M, lo, sg);
        }
        return;
    }
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        const int pidx = a;
        if (Fr::pm(a) == 0) {
            lf[a] = LBM_HPR(own);
        } else {
            const W3 wmar = wsel(-Fr::pm(a), L);
            const float hn = LBM_HPR(nxt);   // 0 beyond a wall
            const float a0 = r.get(0, a), a1 = r.get(1, a);
            lf[a] = fmaf(wmar.p, hn, a0);
            r.set(0, a, fmaf(wmar.z, hn, a1));
            r.set(1, a, wmar.m * hn);
        }
    }
    // transposed wall terms (walls on one axis): the forward adds
    // lambda_+1 f~_a(X) + lambda_-1 f~_abar(X) to f_a(X) for a pointing
    // away from the wall
    const Sides sd = wall_sides<LAT>(G, g, m);
    if (sd.any) {
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            int away = 0, toward = 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int p = sd.s[ax] * Fr::comp(a, ax);
                away += p < 0;
                toward += p > 0;
            }
            if (away) lf[a] = fmaf(L[2], ldb(M, a, own), lf[a]);
            if (toward) lf[a] = fmaf(L[0], ldb(M, La::opp(a), own), lf[a]);
        }
    }
}

template <int LAT, int POL, class NB>
__device__ __forceinline__ void adj_stream_column(const Buf& M, const Buf& O,
                                                  const GatherConst& G, const ColGeom& g, int s,
                                                  const float (&L)[3], int m0, int m1,
                                                  bool inside, const NB& nb) {
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    RevMarch<LAT> r;
    rev_begin<LAT>(M, G, g, s, L, m0, r, nb);
    for (int m = m0; m < m1; ++m) {
        const int mp = nbr(m, 1, G.nm, g.wm);
        const unsigned own = layer_off(g, m);
        const unsigned nxt = layer_off(g, mp);
        float lf[Q];
        rev_layer<LAT>(M, G, g, s, L, m, own, nxt, r, lf, nb);
        if (inside) {
            float lp0 = lf[0];
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                lp0 = fmaf(La::wr(a), lf[a], lp0);
                stb<POL>(O, a, own, lf[a]);
            }
            stb<POL>(O, 0, own, lp0);
        }
    }
}

// The fused reverse step's march over one column: per layer the forward
// gather of f(t) from f~(t-1) (B: the species' view of the state) and the
// reversed gather of the later step's mu (M), then op(P0, F, lam_f, own).
template <int LAT, class NB, class Op>
__device__ __forceinline__ void march_fused(const Buf& B, const Buf& M, const GatherConst& G,
                                            int s, const float (&L)[3], const ColGeom& g, int m0,
                                            int m1, Op& op, const NB& nb, float* macc) {
    constexpr int Q = Lat<LAT>::Q;
    // both marches' partial sums in LDS in 3-D (20 floats per lane each;
    // species 0, the exact shift, has none), which keeps the fused pass at
    // two waves per SIMD for up to four species, and for Op::kThree
    constexpr bool HL = Lat<LAT>::DIM == 3 || Op::kThree;
    Heavy<LAT, HL> h;
    RevMarch<LAT, HL> r;
    if constexpr (HL) {
        h.acc = macc;
        r.acc = macc + 2 * kMarDirs<LAT> * 64;
    }
    if (s > 0) heavy_begin<LAT>(B, G, g, 0, L, m0, h, nb);
    rev_begin<LAT>(M, G, g, s, L, m0, r, nb);
    for (int m = m0; m < m1; ++m) {
        const int mp = nbr(m, 1, G.nm, g.wm);
        const unsigned own = layer_off(g, m);
        const unsigned nxt = layer_off(g, mp);
        float P0, F[Q], lf[Q];
        if (s == 0)
            shift_layer<LAT>(B, G, g, m, own, P0, F);
        else
            heavy_layer<LAT>(B, G, g, 0, L, own, nxt, m, wall_sides<LAT>(G, g, m), h, P0, F,
                             nb);
        rev_layer<LAT>(M, G, g, s, L, m, own, nxt, r, lf, nb);
        op(P0, F, lf, own);
    }
}

#undef LBM_HPR

template <int LAT, int NS, int POL>
__global__ void __launch_bounds__(256) k_adj_stream(const float* __restrict__ mu,
                                                    float* __restrict__ lamout,
                                                    const LatParams* __restrict__ lps,
                                                    const Tile* __restrict__ tiles, int bx) {
    constexpr int DIM = Lat<LAT>::DIM;
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const Tile T = tiles[blockIdx.x];
    const LatParams& P = lps[T.lat];
    // lanes beyond the lattice run along (their neighbours across lanes are
    // the row's last columns) and store nothing
    int x, y;
    bool zero;
    const bool inside = tile_column<LAT>(T, P, lane, bx, x, y, zero);
    const GatherConst G = gather_const(P, DIM);
    ColGeom g = col_geom<LAT>(G, x, y);
    if (zero) g.colbase += kSolid;
    const Buf M = species_buf<LAT>(mu + P.base, P.plane, s);
    const Buf O = species_buf<LAT>(lamout + P.base, P.plane, s);
    const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
    if (bx == 64) {
        const NbWave nb{lane == 0 ? g.col.bxm : (lane == 63 ? g.col.bxp : 0u)};
        adj_stream_column<LAT, POL>(M, O, G, g, s, L, T.m0, T.m1, inside, nb);
    } else {
        adj_stream_column<LAT, POL>(M, O, G, g, s, L, T.m0, T.m1, inside, NbLoad{});
    }
}

// ------------------------------------------------------- fused reverse step
// Kernel B of step t+1 and kernel A of step t in one pass: lam_f(t) = S^T
// mu(t+1) is gathered from the later step's scratch mu (mu_in) where kernel A
// would read lam_s(t); the adjoint stays in population space between the two,
// so the storage transform and its inverse drop out, and mu(t) goes to mu_out.
// The parameter gradients accumulate as in kernel A.
template <int LAT, int NS, int POL>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(AdjSplitOp<LAT, NS, POL>::kThree ? 3 : 1)))
    k_adj_fused(const float* __restrict__ fprev,
                                                   const float* __restrict__ mu_in,
                                                   float* __restrict__ mu_out,
                                                   const LatParams* __restrict__ lps,
                                                   const Tile* __restrict__ tiles, int bx,
                                                   double* __restrict__ gpart) {
    constexpr int DIM = Lat<LAT>::DIM;
    using Op = AdjSplitOp<LAT, NS, POL>;
    __shared__ float x1[NS][4][64];
    __shared__ float x2[NS][Op::KX][64];
    // the two marches' partial sums of every wave (3-D and the three-wave
    // build)
    constexpr bool HL = Lat<LAT>::DIM == 3 || Op::kThree;
    __shared__ float msum[HL ? NS - 1 : 1][HL ? 4 * kMarDirs<LAT> : 1][64];
    __shared__ double gsum[Op::kLdsSums ? NS : 1][Op::NG][64];
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    // (species 0, the exact shift, keeps no marching state)
    float* macc = &msum[HL && s > 0 ? s - 1 : 0][0][lane];
    const Tile T = tiles[blockIdx.x];
    const LatParams& P = lps[T.lat];
    int x, y;
    bool zero;
    const bool inside = tile_column<LAT>(T, P, lane, bx, x, y, zero);
    const Buf M = species_buf<LAT>(mu_in + P.base, P.plane, s);
    // (the op's stored-adjoint view is not read on this path)
    Op op{M, species_buf<LAT>(mu_out + P.base, P.plane, s), coll_const(P), x1, x2, s, lane,
          inside, {}, &gsum[Op::kLdsSums ? s : 0][0][lane]};
#pragma unroll
    for (int q = 0; q < Op::NG; ++q) op.acc(q) = 0.0;
    op.pend = false;
    const GatherConst G = gather_const(P, DIM);
    const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
    ColGeom g = col_geom<LAT>(G, x, y);
    if (zero) g.colbase += kSolid;
    const Buf B = species_buf<LAT>(fprev + P.base, P.plane, s);
    if (bx == 64) {
        const NbWave nb{lane == 0 ? g.col.bxm : (lane == 63 ? g.col.bxp : 0u)};
        march_fused<LAT>(B, M, G, s, L, g, T.m0, T.m1, op, nb, macc);
    } else {
        march_fused<LAT>(B, M, G, s, L, g, T.m0, T.m1, op, NbLoad{}, macc);
    }
    op.flush();
    double sums[Op::NG];
    op.sums(sums);
    block_reduce_add<Op::NG>(sums, gpart + (int64_t)blockIdx.x * Op::NG);
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
    Buf Lb[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) Lb[s] = species_buf<LAT>(lam + P.base, P.plane, s);
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
            float l0 = ldb(Lb[s], 0, own);
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                lt[s][a] = ldb(Lb[s], a, own);
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
static hipError_t adjf_t(const Launch& L, const float* mu_in, float* mu_out, double* gpart) {
    if (L.bx * L.by != 64) return hipErrorInvalidValue;
    auto go = [&](auto pol) {
        hipLaunchKernelGGL((k_adj_fused<LAT, NS, decltype(pol)::value>), dim3(L.ntiles),
                           dim3(64, NS), 0, L.stream, L.src, mu_in, mu_out, L.lp, L.tiles, L.bx,
                           gpart);
    };
    if (L.wt)
        go(std::integral_constant<int, kStoreWT>{});
    else
        go(std::integral_constant<int, kStoreNT>{});
    return hipGetLastError();
}

hipError_t launch_adjoint_fused(int lattice, int ns, const Launch& L, const float* mu_in,
                                float* mu_out, double* gpart) {
    if (lattice == 0) {
        if (ns == 2) return adjf_t<0, 2>(L, mu_in, mu_out, gpart);
        if (ns == 3) return adjf_t<0, 3>(L, mu_in, mu_out, gpart);
        if (ns == 4) return adjf_t<0, 4>(L, mu_in, mu_out, gpart);
    } else {
        if (ns == 2) return adjf_t<1, 2>(L, mu_in, mu_out, gpart);
        if (ns == 3) return adjf_t<1, 3>(L, mu_in, mu_out, gpart);
        if (ns == 4) return adjf_t<1, 4>(L, mu_in, mu_out, gpart);
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
