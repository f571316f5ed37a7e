// Forward kernels: the fused time step, the initial state, and the
// observables with their FP64 reductions, with launchers templated on the
// lattice.  Each lattice is compiled in its own translation unit
// (step_d2q9.hip, step_d3q19.hip); step.hip dispatches between them.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "collide.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace lbmmc {

// Work-groups are dealt to the eight XCDs round-robin by work-group id.  Map
// the id to a "virtual" id so that the work-groups on one XCD take a
// contiguous range of the (spatially ordered) tile list and share its halo
// rows in their XCD's L2.  Bijective for any grid size.
__device__ __forceinline__ void tile_range(int ntiles, int& t0, int& t1) {
    const int G = gridDim.x, b = blockIdx.x;
    const int k = b & 7, idx = b >> 3, per = G >> 3, rem = G & 7;
    const int vb = k * per + (k < rem ? k : rem) + idx;
    if (G == ntiles) {
        // one tile per work-group (every non-persistent launch): the 64-bit
        // divisions below are a long scalar sequence at the start of every
        // wave, 0.1 us of a 6.2 us step on a small lattice
        t0 = vb;
        t1 = vb + 1;
        return;
    }
    t0 = (int)((int64_t)vb * ntiles / G);
    t1 = (int)((int64_t)(vb + 1) * ntiles / G);
}

// Index of node (x, y, layer m) in the dense node fields of a lattice.
template <int LAT>
__device__ __forceinline__ int64_t dense_node(const LatParams& P, int x, int y, int m) {
    return Lat<LAT>::DIM == 2 ? (int64_t)m * P.nx + x : ((int64_t)m * P.ny + y) * P.nx + x;
}

// Specific force at a node: the constant g, or (KF) the caller's force field
// k(x), dense node fields [lattice][d][nodes] (d = 2 or 3 components).
template <int LAT, bool KF>
__device__ __forceinline__ void node_accel(const float* accel, const LatParams& P, const float* gc,
                                           int64_t node, float (&g)[3]) {
    constexpr int DIM = Lat<LAT>::DIM;
    if constexpr (KF) {
        const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
        const float* a = accel + P.field_base * DIM;
        g[0] = a[node];
        g[1] = a[nodes + node];
        g[2] = DIM == 3 ? a[2 * nodes + node] : 0.0f;
    } else {
        g[0] = gc[0];
        g[1] = gc[1];
        g[2] = gc[2];
    }
}

// Density gradients of every species at node (x, y, layer m) from the dense
// density fields of one lattice (FRC 2).
template <int LAT, int NS>
__device__ __forceinline__ void species_grads(const float* dens, const LatParams& P, int x, int y,
                                              int m, float (&gi)[NS][3]) {
    constexpr int DIM = Lat<LAT>::DIM;
    const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const float* f = dens + s * nodes;
        field_grad<DIM>([&](int64_t j) { return f[j]; }, P.nx, P.ny, P.nz, P.wall_mask, x,
                        DIM == 2 ? m : y, DIM == 2 ? 0 : m, gi[s]);
    }
}

template <int LAT, int NS, int FRC, int EXT, int POL>
struct StepOp {
    static constexpr int Q = Lat<LAT>::Q;
    Buf D[NS];               // the destination's species views
    CollConst C;
    bool bad;
    const float* dens;      // FRC 2: this lattice's density fields
    const LatParams* P;
    int x, y;
    const float* accel;     // EXT 1: the force field
    __device__ __forceinline__ void operator()(float (&P0)[NS], float (&F)[NS][Q], int m,
                                               unsigned own) {
        float gi[NS][3] = {};
        if constexpr (FRC == 2) species_grads<LAT, NS>(dens, *P, x, y, m, gi);
        float g[3];
        node_accel<LAT, EXT == 1>(accel, *P, C.g, dense_node<LAT>(*P, x, y, m), g);
        constexpr int DIM = Lat<LAT>::DIM;
        WallMove W{};
        const bool mw = EXT == 2 && moving_wall_at(*P, x, DIM == 2 ? m : y, DIM == 2 ? 0 : m, W);
        if (!collide<LAT, NS, FRC>(P0, F, C, g, gi, mw, W)) bad = true;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            stb<POL>(D[s], 0, own, P0[s]);
#pragma unroll
            for (int a = 1; a < Q; ++a) stb<POL>(D[s], a, own, F[s][a]);
        }
    }
};

template <int LAT, int NS, int FRC, int EXT, int POL>
__global__ void __launch_bounds__(256) k_step(const float* __restrict__ src, float* __restrict__ dst,
                                              const LatParams* __restrict__ lps,
                                              const Tile* __restrict__ tiles, int ntiles,
                                              const float* __restrict__ dens,
                                              const float* __restrict__ accel,
                                              unsigned* __restrict__ flag) {
    constexpr int DIM = Lat<LAT>::DIM;
    int t0, t1;
    tile_range(ntiles, t0, t1);
    bool bad = false;
    for (int t = t0; t < t1; ++t) {
        const Tile T = tiles[t];
        const LatParams& P = lps[T.lat];
        const int x = T.x0 + (int)threadIdx.x;
        const int y = DIM == 3 ? T.y0 + (int)threadIdx.y : 0;
        if (x >= P.nx || (DIM == 3 && y >= P.ny)) continue;
        const GatherConst G = gather_const(P, DIM);
        StepOp<LAT, NS, FRC, EXT, POL> op{{}, coll_const(P), false,
                                    FRC == 2 ? dens + P.field_base * NS : nullptr, &P, x, y,
                                    accel};
        Buf B[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            B[s] = species_buf<LAT>(src + P.base, P.plane, s);
            op.D[s] = species_buf<LAT>(dst + P.base, P.plane, s);
        }
        march<LAT, NS, EXT == 3>(B, G, x, y, T.m0, T.m1, op);
        bad = bad || op.bad;
    }
    if (bad) atomicOr(flag, 1u);
}

// ------------------------------------------------------ species-split step
// The same fused step with one wavefront per species: a work-group is NS
// waves over the same 64 cross-section columns, wave s gathers species s
// only, the waves exchange each node's (rho_s, u_s^eq) through LDS
// (double-buffered, one barrier per layer), and each wave then forms the
// mixture and the cross relaxation (identical arithmetic in every wave) and
// collides and stores its own species.  A wave holds one species' marching
// state instead of NS, and keeps its marching-axis partial sums in LDS
// (2 per direction with a marching component: 12 floats per lane in 2-D, 20
// in 3-D; see kSplitLdsMarch), so several times more waves fit on a SIMD:
// five in 2-D, four in 3-D (three with the sums in registers).
//
// A work-group may hold W such segments of 64 columns side by side
// (threadIdx.z = segment; bx * by = 64 W): W consecutive 64-column pieces of
// an x row in 2-D, W consecutive y rows of 64 columns in 3-D.  All NS x W
// waves march the same layers in step (the per-layer barrier), so the
// neighbour columns one segment reads at its edges (x halo in 2-D) or the
// neighbour rows it reads across (y +- 1 in 3-D) are the rows its sibling
// segments load in the same layer: they come from the caches instead of
// memory, and only the work-group's outer halo is fetched twice.
template <int LAT, int NS, int FRC, int EXT, int POL>
struct SplitOp {
    static constexpr int Q = Lat<LAT>::Q;
    Buf D;
    CollConst C;
    SpeciesConst K;
    float4* xch;             // [2][W][NS][64] exchange buffers in LDS
    float4* xgr;             // FRC 2: [2][W][NS][64] exchange of the density gradients
    int xstride;             // W * NS * 64: floats4 per exchange buffer
    int s, lane;
    bool inside, bad;
    const float* dens;       // FRC 2: this species' density field
    const LatParams* P;
    int x, y;
    const float* accel;      // EXT 1: the force field
    // 2-D: the stores of layer m are issued in the next layer's call, after
    // that layer's gather has its loads back.  A wave's vector memory counter
    // retires in issue order, so stores issued just before the next layer's
    // loads would hold the first wait on those loads until the stores are
    // acknowledged; issued later, their completion overlaps the exchange
    // barrier and the collision (bit-identical, about 2 % faster per step).
    // In 3-D they are stored at once: deferred, the step measured far slower.
    static constexpr bool kDefer = Lat<LAT>::DIM == 2;
    float out[Q];            // kDefer: the pending layer's values
    unsigned out_own;
    bool pend;
    __device__ __forceinline__ void flush() {
        if (pend) {
#pragma unroll
            for (int a = 0; a < Q; ++a) stb<POL>(D, a, out_own, out[a]);
        }
        pend = false;
    }
    __device__ __forceinline__ void operator()(float P0, float (&F)[Q], int m, unsigned own) {
        constexpr int DIM = Lat<LAT>::DIM;
        if constexpr (kDefer) flush();
        float g[3];
        node_accel<LAT, EXT == 1>(accel, *P, C.g, dense_node<LAT>(*P, x, y, m), g);
        float rho_s, dlt_s, ue_s[3];
        species_moments<LAT>(P0, F, K.c, g, rho_s, dlt_s, ue_s);
        float4* X = xch + (m & 1) * xstride;
        X[s * 64 + lane] = make_float4(rho_s, ue_s[0], ue_s[1], ue_s[2]);
        Grads gd{};
        if constexpr (FRC == 2) {
            const float* f = dens;
            field_grad<DIM>([&](int64_t j) { return f[j]; }, P->nx, P->ny, P->nz, P->wall_mask,
                            x, DIM == 2 ? m : y, DIM == 2 ? 0 : m, gd.gi);
            xgr[(m & 1) * xstride + s * 64 + lane] =
                make_float4(gd.gi[0], gd.gi[1], gd.gi[2], 0.0f);
        }
        __syncthreads();
        if constexpr (FRC == 2) {
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const float4 v = xgr[(m & 1) * xstride + j * 64 + lane];
                gd.gm[0] += v.x;
                gd.gm[1] += v.y;
                gd.gm[2] += v.z;
            }
        }
        float rho[NS], ue[NS][3];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const float4 v = X[j * 64 + lane];
            rho[j] = v.x;
            ue[j][0] = v.y;
            ue[j][1] = v.z;
            ue[j][2] = v.w;
        }
        WallMove W{};
        if (EXT == 2 && moving_wall_at(*P, x, DIM == 2 ? m : y, DIM == 2 ? 0 : m, W)) {
            wall_shift_ue<NS>(W, rho, ue);
            float R = 0.0f;
#pragma unroll
            for (int j = 0; j < NS; ++j) R += rho[j];
            wall_add_terms<LAT>(W, rho_s, rho_s * rcp_nr(R), K.c, F);
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                if (i != s) continue;
                ue_s[0] = ue[i][0];
                ue_s[1] = ue[i][1];
                ue_s[2] = ue[i][2];
            }
        }
        const Mix M = mixture<NS>(rho, ue, C);
        float y[NS][NS];
        tau_solve<NS>(rho, M.R, M.n, C, y);
        // friction of the own species (s is uniform over the wave)
        float V[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i != s) continue;
            friction<NS>(i, rho, ue, y, M.iR, V);
        }
        const bool ok = collide_species<LAT, FRC>(K, g, rho_s, dlt_s, ue_s, M, V, gd, P0, F) &&
                        isfinite(M.R);
        if (inside) {
            if constexpr (kDefer) {
                out[0] = P0;
#pragma unroll
                for (int a = 1; a < Q; ++a) out[a] = F[a];
                out_own = own;
                pend = true;
            } else {
                stb<POL>(D, 0, own, P0);
#pragma unroll
                for (int a = 1; a < Q; ++a) stb<POL>(D, a, own, F[a]);
            }
            bad = bad || !ok;
        }
    }
};

// Where the species-split step keeps its marching partial sums: in LDS,
// except for 2-D states held in the last-level cache (written-through
// stores), where one tile's chain sets the step time and registers are
// faster (6.23 against 6.31 us per step on the 1024x64 tube).
template <int LAT, int POL>
constexpr bool kSplitLdsMarch = Lat<LAT>::DIM == 3 || POL != kStoreWT;

// Work-group size limit of the species-split kernels: NS x W waves of 64
// lanes with W <= 4 and NS x W <= 12 (three waves per SIMD).
constexpr int kSplitMaxThreads = 768;

template <int LAT, int NS, int FRC, int EXT, int POL>
__global__ void __launch_bounds__(kSplitMaxThreads) k_step_split(
        const float* __restrict__ src, float* __restrict__ dst,
        const LatParams* __restrict__ lps, const Tile* __restrict__ tiles, int ntiles, int bx,
        const float* __restrict__ dens, const float* __restrict__ accel,
        unsigned* __restrict__ flag) {
    constexpr int DIM = Lat<LAT>::DIM;
    // [FRC == 2 ? 2 : 1][2][W][NS][64] float4: the exchange buffers (and those
    // of the density gradients), sized by the launch
    extern __shared__ float4 smem[];
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int seg = __builtin_amdgcn_readfirstlane((int)threadIdx.z);
    const int W = (int)blockDim.z;
    const int xstride = W * NS * 64;
    float4* xch = smem + seg * NS * 64;
    float4* xgr = smem + 2 * xstride + seg * NS * 64;
    // this wave's marching partial sums (when kept in LDS), after the
    // exchange buffers
    float* macc = reinterpret_cast<float*>(smem + (FRC == 2 ? 2 : 1) * 2 * xstride) +
                  (seg * NS + s) * 2 * kMarDirs<LAT> * 64 + lane;
    int t0, t1;
    tile_range(ntiles, t0, t1);
    bool bad = false;
    for (int t = t0; t < t1; ++t) {
        const Tile T = tiles[t];
        const LatParams& P = lps[T.lat];
        // lanes beyond the lattice still run (every wave must reach the
        // barriers) and store nothing
        int x, y;
        bool zero;
        const bool inside = tile_column_seg<LAT>(T, P, lane, bx, seg, W, x, y, zero);
        const GatherConst G = gather_const(P, DIM);
        // the species' own constants, read with the uniform species index
        // (scalar loads; no run-time indexing of register arrays)
        const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
        SplitOp<LAT, NS, FRC, EXT, POL> op{species_buf<LAT>(dst + P.base, P.plane, s),
                                 coll_const(P),
                                 SpeciesConst{P.c[s], P.inv_cs2[s], P.inv_tau[s], P.fpref[s],
                                              P.kdiff[s], P.cs2[s]},
                                 xch, xgr, xstride, s, lane, inside, false,
                                 FRC == 2 ? dens + P.field_base * NS
                                                + s * ((int64_t)P.nx * P.ny * P.nz)
                                          : nullptr,
                                 &P, x, y, accel, {}, 0u, false};
        march1<LAT, decltype(op), kSplitLdsMarch<LAT, POL>>(
                species_buf<LAT>(src + P.base, P.plane, s), G, s, L, x, y, zero, bx % 64 == 0,
                T.m0, T.m1, op, macc);
        op.flush();
        bad = bad || op.bad;
        __syncthreads();   // the next tile reuses the exchange buffers
    }
    if (bad) atomicOr(flag, 1u);
}

// ------------------------------------------------- density pre-pass (FRC 2)
// The pressure and density forcing contributions need density gradients at
// the time level of the collision, i.e. the densities of the streamed
// populations at the neighbours.  This pass streams every node (the same
// gather as the fused step) and stores rho_s = P0/w_0 + sum_a F_a into dense
// node fields [N][nodes]; the fused step then reads the neighbours' values.
template <int LAT>
__device__ __forceinline__ float streamed_density(float P0, const float (&F)[Lat<LAT>::Q]) {
    float sf = 0.0f;
#pragma unroll
    for (int a = 1; a < Lat<LAT>::Q; ++a) sf += F[a];
    return fmaf(P0, Lat<LAT>::inv_w0, sf);
}

template <int LAT, int NS>
struct DensOp {
    static constexpr int Q = Lat<LAT>::Q;
    float* out;
    const LatParams* P;
    int64_t nodes;
    int x, y;
    __device__ __forceinline__ void operator()(float (&P0)[NS], float (&F)[NS][Q], int m,
                                               unsigned) {
        const int64_t node = dense_node<LAT>(*P, x, y, m);
#pragma unroll
        for (int s = 0; s < NS; ++s) out[s * nodes + node] = streamed_density<LAT>(P0[s], F[s]);
    }
};

template <int LAT>
struct DensOp1 {
    static constexpr int Q = Lat<LAT>::Q;
    float* out;               // this species' field
    const LatParams* P;
    int x, y;
    bool inside;
    __device__ __forceinline__ void operator()(float P0, float (&F)[Q], int m, unsigned) {
        const float r = streamed_density<LAT>(P0, F);
        if (inside) out[dense_node<LAT>(*P, x, y, m)] = r;
    }
};

template <int LAT, int NS>
__global__ void __launch_bounds__(256) k_density(const float* __restrict__ src,
                                                 const LatParams* __restrict__ lps,
                                                 const Tile* __restrict__ tiles, int ntiles,
                                                 float* __restrict__ dens) {
    constexpr int DIM = Lat<LAT>::DIM;
    int t0, t1;
    tile_range(ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const Tile T = tiles[t];
        const LatParams& P = lps[T.lat];
        const int x = T.x0 + (int)threadIdx.x;
        const int y = DIM == 3 ? T.y0 + (int)threadIdx.y : 0;
        if (x >= P.nx || (DIM == 3 && y >= P.ny)) continue;
        const GatherConst G = gather_const(P, DIM);
        const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
        DensOp<LAT, NS> op{dens + P.field_base * NS, &P, nodes, x, y};
        Buf B[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) B[s] = species_buf<LAT>(src + P.base, P.plane, s);
        march<LAT, NS>(B, G, x, y,
                       T.m0, T.m1, op);
    }
}

// species-split form: block (64, NS, W), wave (s, seg) streams species s on
// segment seg of the tile
template <int LAT, int NS>
__global__ void __launch_bounds__(kSplitMaxThreads) k_density_split(
        const float* __restrict__ src, const LatParams* __restrict__ lps,
        const Tile* __restrict__ tiles, int ntiles, int bx, float* __restrict__ dens) {
    constexpr int DIM = Lat<LAT>::DIM;
    const int lane = (int)threadIdx.x;
    const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int seg = __builtin_amdgcn_readfirstlane((int)threadIdx.z);
    const int W = (int)blockDim.z;
    int t0, t1;
    tile_range(ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const Tile T = tiles[t];
        const LatParams& P = lps[T.lat];
        int x, y;
        bool zero;
        const bool inside = tile_column_seg<LAT>(T, P, lane, bx, seg, W, x, y, zero);
        const GatherConst G = gather_const(P, DIM);
        const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
        const float L[3] = {P.lam[s][0], P.lam[s][1], P.lam[s][2]};
        DensOp1<LAT> op{dens + P.field_base * NS + s * nodes, &P, x, y, inside};
        march1<LAT>(species_buf<LAT>(src + P.base, P.plane, s), G, s, L, x, y, zero,
                    bx % 64 == 0, T.m0, T.m1, op);
    }
}

// Initial state of one lattice: f(0) = [1 + e.u_i0/c_s^2] omega rho_i with
// u_i0 = -g/2 (force-consistent initial velocity, zero species and mixture
// velocity), rho_i = x_i M_i n0, evaluated in double and stored as
// P0 = f_0 and g_a = f_a - (w_a/w_0) P0 + w_a (f_0 - P0)/(1 - w_0) in f0_out;
// then one collision, stored in ft_out.
template <int LAT, int NS, int FRC, int EXT>
__global__ void __launch_bounds__(256) k_init(const LatParams* __restrict__ lps, int lat,
                                              const double* __restrict__ x0,
                                              const float* __restrict__ accel,
                                              float* __restrict__ f0_out,
                                              float* __restrict__ ft_out,
                                              unsigned* __restrict__ flag) {
    constexpr int Q = Lat<LAT>::Q;
    const LatParams& P = lps[lat];
    const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
    const double* xl = x0 + P.field_base * NS;
    const CollConst C = coll_const(P);
    bool bad = false;
    const double w0 = LAT == 0 ? 4.0 / 9.0 : 1.0 / 3.0;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < nodes;
         id += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(id % P.nx);
        const int64_t r = id / P.nx;
        const int y = (int)(r % P.ny);
        const int z = (int)(r / P.ny);
        const int64_t own = P.base + ((int64_t)z * P.ny + y) * P.pitch + x;
        float g[3];
        node_accel<LAT, EXT == 1>(accel, P, C.g, id, g);
        float P0[NS], F[NS][Q];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double rho = xl[s * nodes + id] * (double)P.M[s] * (double)P.n0;
            const double c = (double)C.c[s], ics = (double)C.inv_cs2[s];
            const double f0 = w0 * rho;
            const float p0 = (float)f0;
            const double rem = (f0 - (double)p0) / (1.0 - w0);
            P0[s] = p0;
            F[s][0] = 0.0f;
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const double wa = LAT == 0 ? (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0)
                                           : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
                const double eu = c * (double)cdot<LAT>(a, -0.5f * g[0], -0.5f * g[1],
                                                        -0.5f * g[2]);
                const double fa = wa * rho * (1.0 + ics * eu);
                F[s][a] = (float)(fa - wa / w0 * (double)p0 + wa * rem);
            }
            f0_out[(int64_t)(s * Q) * P.plane + own] = p0;
#pragma unroll
            for (int a = 1; a < Q; ++a) f0_out[(int64_t)(s * Q + a) * P.plane + own] = F[s][a];
        }
        // f(0) as gather output: P0 and F_a = f_a - w_a r* = g_a
        float gi[NS][3] = {};
        if constexpr (FRC == 2) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const double sc = (double)P.M[s] * (double)P.n0;
                const double* xs = xl + s * nodes;
                field_grad<Lat<LAT>::DIM>([&](int64_t j) { return (float)(xs[j] * sc); }, P.nx,
                                          P.ny, P.nz, P.wall_mask, x, y, z, gi[s]);
            }
        }
        if (!collide<LAT, NS, FRC>(P0, F, C, g, gi, false, WallMove{}))   // f(0): not streamed
            bad = true;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            ft_out[(int64_t)(s * Q) * P.plane + own] = P0[s];
#pragma unroll
            for (int a = 1; a < Q; ++a) ft_out[(int64_t)(s * Q + a) * P.plane + own] = F[s][a];
        }
    }
    if (bad) atomicOr(flag, 1u);
}

// ------------------------------------------------------------- observables
template <int LAT, int NS>
struct MomOp {
    static constexpr int Q = Lat<LAT>::Q;
    static constexpr int DIM = Lat<LAT>::DIM;
    float* rho_out;
    float* x_out;
    float* u_out;
    float* ueq_out;          // [N][d][nodes]: u_i^eq
    float* us_out;           // [N][d][nodes]: u_i = u_i^eq - Theta_i/(2 rho_i)
    int64_t nodes;
    int nx, ny, x, y;
    CollConst C;
    const float* accel;      // this lattice's force field, or null (constant g)
    const LatParams* P;
    bool streamed;           // the populations come from a stream (not f(0))
    double acc[NS + 3];
    __device__ __forceinline__ void operator()(float (&P0)[NS], float (&F)[NS][Q], int m,
                                               unsigned) {
        const int64_t node = DIM == 2 ? (int64_t)m * nx + x : ((int64_t)m * ny + y) * nx + x;
        float g[3] = {C.g[0], C.g[1], C.g[2]};
        if (accel) {
            g[0] = accel[node];
            g[1] = accel[nodes + node];
            g[2] = DIM == 3 ? accel[2 * nodes + node] : 0.0f;
        }
        float rho[NS], dlt[NS], ue[NS][3];
#pragma unroll
        for (int s = 0; s < NS; ++s)
            species_moments<LAT>(P0[s], F[s], C.c[s], g, rho[s], dlt[s], ue[s]);
        WallMove W;
        if (streamed && moving_wall_at(*P, x, DIM == 2 ? m : y, DIM == 2 ? 0 : m, W))
            wall_shift_ue<NS>(W, rho, ue);
        float R = 0.0f, n = 0.0f, U[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            R += rho[s];
            n += rho[s] * C.invM[s];
#pragma unroll
            for (int d = 0; d < 3; ++d) U[d] = fmaf(rho[s], ue[s][d], U[d]);
        }
        const float iR = 1.0f / R;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (rho_out) rho_out[s * nodes + node] = rho[s];
            if (x_out) x_out[s * nodes + node] = rho[s] * C.invM[s] / n;
            acc[s] += (double)rho[s];
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (u_out) u_out[d * nodes + node] = U[d] * iR;
            acc[NS + d] += (double)U[d];   // rho u = sum_i rho_i u_i^eq
        }
        if (ueq_out) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int d = 0; d < DIM; ++d) ueq_out[(s * DIM + d) * nodes + node] = ue[s][d];
        }
        if (us_out) {
            // eq. (CE_EQ83) with Theta_i of eq. (CE_theta_definition):
            // Theta_i/rho_i = sum_j rho_j/(rho tau_ij) (u_i^eq - u_j^eq), the
            // friction vector V_i of the collision (its limit where rho_i = 0)
            const Mix Mx = mixture<NS>(rho, ue, C);
            float y[NS][NS];
            tau_solve<NS>(rho, Mx.R, Mx.n, C, y);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                float V[3];
                friction<NS>(s, rho, ue, y, Mx.iR, V);
#pragma unroll
                for (int d = 0; d < DIM; ++d)
                    us_out[(s * DIM + d) * nodes + node] = fmaf(-0.5f, V[d], ue[s][d]);
            }
        }
    }
};

template <int LAT, int NS, bool EQ>
__global__ void __launch_bounds__(256) k_moments(const float* __restrict__ src,
                                                 const LatParams* __restrict__ lps,
                                                 const Tile* __restrict__ tiles, int direct,
                                                 const float* __restrict__ accel,
                                                 float* rho, float* xo, float* u, float* ueq,
                                                 float* us, double* __restrict__ partial,
                                                 int nq) {
    constexpr int Q = Lat<LAT>::Q;
    constexpr int DIM = Lat<LAT>::DIM;
    __shared__ double red[4][NS + 3];
    const int t = blockIdx.x;
    const Tile T = tiles[t];
    const LatParams& P = lps[T.lat];
    const int x = T.x0 + (int)threadIdx.x;
    const int y = DIM == 3 ? T.y0 + (int)threadIdx.y : 0;
    const int64_t nodes = (int64_t)P.nx * P.ny * P.nz;
    MomOp<LAT, NS> op;
    op.rho_out = rho ? rho + P.field_base * NS : nullptr;
    op.x_out = xo ? xo + P.field_base * NS : nullptr;
    op.u_out = u ? u + P.field_base * DIM : nullptr;
    op.ueq_out = ueq ? ueq + P.field_base * NS * DIM : nullptr;
    op.us_out = us ? us + P.field_base * NS * DIM : nullptr;
    op.nodes = nodes;
    op.nx = P.nx; op.ny = P.ny; op.x = x; op.y = y;
    op.C = coll_const(P);
    op.accel = accel ? accel + P.field_base * DIM : nullptr;
    op.P = &P;
    op.streamed = !direct;
#pragma unroll
    for (int q = 0; q < NS + 3; ++q) op.acc[q] = 0.0;
    if (x < P.nx && (DIM == 2 || y < P.ny)) {
        const float* lb = src + P.base;
        if (direct) {
            for (int m = T.m0; m < T.m1; ++m) {
                const int64_t own = (DIM == 2 ? (int64_t)m * P.pitch : ((int64_t)m * P.ny + y) * P.pitch) + x;
                float P0[NS], F[NS][Q];
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    P0[s] = lb[(int64_t)(s * Q) * P.plane + own];
                    F[s][0] = 0.0f;
#pragma unroll
                    for (int a = 1; a < Q; ++a) F[s][a] = lb[(int64_t)(s * Q + a) * P.plane + own];
                }
                op(P0, F, m, 0u);
            }
        } else {
            const GatherConst G = gather_const(P, DIM);
            Buf B[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) B[s] = species_buf<LAT>(lb, P.plane, s);
            march<LAT, NS, EQ>(B, G, x, y, T.m0, T.m1, op);
        }
    }
    // block reduction: wave shuffles, then the waves in a fixed order
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wave = tid >> 6;
    const int nwaves = (blockDim.x * blockDim.y + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NS + DIM; ++q) {
        double v = op.acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (tid < NS + DIM) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[w][tid];
        partial[(int64_t)t * nq + tid] = s;
    }
}

// ---------------------------------------------------------------- launchers
// Calls fn(lattice, species count, forcing, extension) with the four as
// compile-time constants; extension 0: constant g and resting walls, 1: a
// force field, 2: moving walls, 3: the equilibrium comparison boundary.
template <int LAT, typename Fn>
static hipError_t by_shape(int ns, int frc, int ext, Fn&& fn) {
    using std::integral_constant;
    constexpr integral_constant<int, LAT> lat{};
    auto with_ext = [&](auto n, auto f) -> hipError_t {
        if (ext == 0) return fn(lat, n, f, integral_constant<int, 0>{});
        if (ext == 1) return fn(lat, n, f, integral_constant<int, 1>{});
        if (ext == 2) return fn(lat, n, f, integral_constant<int, 2>{});
        if (ext == 3) return fn(lat, n, f, integral_constant<int, 3>{});
        return hipErrorInvalidValue;
    };
    auto with_frc = [&](auto n) -> hipError_t {
        if (frc == 0) return with_ext(n, integral_constant<int, 0>{});
        if (frc == 1) return with_ext(n, integral_constant<int, 1>{});
        if (frc == 2) return with_ext(n, integral_constant<int, 2>{});
        return hipErrorInvalidValue;
    };
    if (ns == 2) return with_frc(integral_constant<int, 2>{});
    if (ns == 3) return with_frc(integral_constant<int, 3>{});
    if (ns == 4) return with_frc(integral_constant<int, 4>{});
    return hipErrorInvalidValue;
}

template <int LAT_>
hipError_t launch_step_lat(int ns, const Launch& L) {
    if (L.split && !split_shape_ok(L.bx, L.by, ns)) return hipErrorInvalidValue;
    return by_shape<LAT_>(ns, L.forcing, L.eqb ? 3 : (L.accel ? 1 : (L.moving ? 2 : 0)),
                    [&](auto lat, auto n, auto frc, auto ex) -> hipError_t {
        constexpr int LAT = decltype(lat)::value, NS = decltype(n)::value,
                      FRC = decltype(frc)::value, EXT = decltype(ex)::value;
        // the fused step with the store policy the host chose (a template
        // argument: the policy is an immediate of the store instructions)
        auto step = [&](auto pol) -> hipError_t {
            constexpr int POL = decltype(pol)::value;
            if constexpr (EXT != 3) {   // (the equilibrium boundary has no split form)
                if (L.split) {
                    const int W = L.bx * L.by / 64;
                    const size_t lds = (FRC == 2 ? 2 : 1) * 2 * (size_t)W * NS * 64 * sizeof(float4) +
                                       (kSplitLdsMarch<LAT, POL>
                                            ? (size_t)W * NS * 2 * kMarDirs<LAT> * 64 * sizeof(float)
                                            : 0);
                    hipLaunchKernelGGL((k_step_split<LAT, NS, FRC, EXT, POL>), dim3(L.grid),
                                       dim3(64, NS, W), lds, L.stream, L.src, L.dst, L.lp,
                                       L.tiles, L.ntiles, L.bx, L.dens, L.accel, L.flag);
                    return hipGetLastError();
                }
            }
            hipLaunchKernelGGL((k_step<LAT, NS, FRC, EXT, POL>), dim3(L.grid), dim3(L.bx, L.by),
                               0, L.stream, L.src, L.dst, L.lp, L.tiles, L.ntiles, L.dens,
                               L.accel, L.flag);
            return hipGetLastError();
        };
        if constexpr (EXT == 3) {
            // the equilibrium boundary: standard forcing, one thread per column
            if constexpr (FRC != 0) {
                return hipErrorInvalidValue;
            } else {
                if (L.split) return hipErrorInvalidValue;
                return L.wt ? step(std::integral_constant<int, kStoreWT>{})
                            : step(std::integral_constant<int, kStoreNT>{});
            }
        } else {
            if (FRC == 2) {
                if (!L.dens) return hipErrorInvalidValue;
                // (the force does not enter the densities)
                if (L.split)
                    hipLaunchKernelGGL((k_density_split<LAT, NS>), dim3(L.grid),
                                       dim3(64, NS, L.bx * L.by / 64), 0, L.stream, L.src, L.lp,
                                       L.tiles, L.ntiles, L.bx, L.dens);
                else
                    hipLaunchKernelGGL((k_density<LAT, NS>), dim3(L.grid), dim3(L.bx, L.by), 0,
                                       L.stream, L.src, L.lp, L.tiles, L.ntiles, L.dens);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
            }
            return L.wt ? step(std::integral_constant<int, kStoreWT>{})
                        : step(std::integral_constant<int, kStoreNT>{});
        }
    });
}

template <int LAT_>
hipError_t launch_init_lat(int ns, const LatParams* lp, int lat, const LatParams& h,
                           const double* x0, const float* accel, float* f0, float* ft,
                           unsigned* flag, hipStream_t s) {
    const int64_t nodes = (int64_t)h.nx * h.ny * h.nz;
    const int64_t blocks = std::min<int64_t>((nodes + 255) / 256, 65536);
    // the initial collision acts on f(0), which has not been streamed: no wall terms
    return by_shape<LAT_>(ns, h.forcing, accel ? 1 : 0,
                    [&](auto la, auto n, auto frc, auto ex) {
        constexpr int LAT = decltype(la)::value, NS = decltype(n)::value,
                      FRC = decltype(frc)::value, EXT = decltype(ex)::value;
        if constexpr (EXT >= 2) {
            return hipErrorInvalidValue;   // (not requested: no streaming at init)
        } else {
            hipLaunchKernelGGL((k_init<LAT, NS, FRC, EXT>), dim3((unsigned)blocks), dim3(256), 0,
                               s, lp, lat, x0, accel, f0, ft, flag);
            return hipGetLastError();
        }
    });
}

template <int LAT, int NS>
static hipError_t launch_moments_t(const Launch& L, int direct, float* rho, float* x, float* u,
                                   float* ueq, float* us, double* partial, int nq) {
    if (L.eqb)
        hipLaunchKernelGGL((k_moments<LAT, NS, true>), dim3(L.ntiles), dim3(L.bx, L.by), 0,
                           L.stream, L.src, L.lp, L.tiles, direct, L.accel, rho, x, u, ueq, us,
                           partial, nq);
    else
        hipLaunchKernelGGL((k_moments<LAT, NS, false>), dim3(L.ntiles), dim3(L.bx, L.by), 0,
                           L.stream, L.src, L.lp, L.tiles, direct, L.accel, rho, x, u, ueq, us,
                           partial, nq);
    return hipGetLastError();
}

template <int LAT>
hipError_t launch_moments_lat(int ns, const Launch& L, int direct, float* rho, float* x,
                              float* u, float* ueq, float* us, double* partial, int nq) {
    if (ns == 2) return launch_moments_t<LAT, 2>(L, direct, rho, x, u, ueq, us, partial, nq);
    if (ns == 3) return launch_moments_t<LAT, 3>(L, direct, rho, x, u, ueq, us, partial, nq);
    if (ns == 4) return launch_moments_t<LAT, 4>(L, direct, rho, x, u, ueq, us, partial, nq);
    return hipErrorInvalidValue;
}

}  // namespace lbmmc
