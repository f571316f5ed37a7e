// Device building blocks of the fused step: the pull gather (streaming with
// the second-order interpolation and the impermeable-wall scheme).
//
// Storage.  Per species and node the state is kept as
//     plane 0:       P0 = f~_0                                (rest population)
//     plane a >= 1:  g_a = f~_a - (w_a/w_0) P0                (deviation from rest)
// i.e. the populations relative to the rest state of reference density
// r* = P0/w_0; the species density is rho = r* + sum_{a>=1} g_a.  This is the
// same information as the Q post-collision populations in the same number of
// floats, but the small deviations carry the low-order bits: the mass and the
// momentum -- small differences of O(rho) numbers in the plain representation
// -- are kept to FP32 precision of the deviations, not of rho (when P0 is
// rounded on store, its rounding error is moved isotropically into the g_a,
// so no mass is lost).  The gather never forms an O(rho) population: the
// reference part of a streamed population enters only through differences
// P0(O+k) - P0(O), which are exact or nearly so.
//
// Gather.  A work-group owns a block of cross-section columns (x in 2-D,
// (x, y) in 3-D); each thread owns one column and marches through layers
// [m0, m1) of the slowest axis (y in 2-D, z in 3-D).  The interpolation of
// eq. (Second_order_spatial_interpolation) is a product of 1-D quadratic
// Lagrange factors, applied as nested 1-D passes: the cross-section passes
// read neighbouring columns straight from memory (L1/L2 hits: the
// neighbouring lanes of the same instruction read the same rows), and the
// pass along the marching axis is carried in registers (two running partial
// sums per deviation plane, three layers of the reference stencil), so every
// value of a layer is fetched from HBM about once.  Species 1 (c = 1) is an
// exact one-node shift.
//
// Addressing.  Loads and stores are buffer instructions: one buffer resource
// per species of a lattice (scalar registers), the direction plane as a
// scalar byte offset and the node as a 32-bit per-lane byte offset, so no
// per-load 64-bit address arithmetic is needed (each species' Q planes stay
// below 2 GiB; a buffer holds up to 4 of them).
//
// For every node the gather hands over, per species s:
//   P0[s]     the stored rest population at the node (it does not stream),
//   F[s][a]   f_a(O) - w_a r*(O) for a >= 1, f_a the streamed population.
// With the FP32 weight triples summing to exactly 1 and the wall terms handing
// back the stored weights that a solid layer would have received (Appendix A),
// the update moves mass without systematic drift.
#pragma once

#include "common.hpp"
#include "lattice.hpp"

namespace lbmmc {

// Buffer view of the Q planes of one species of a lattice (plane a of the view
// is direction a of that species).
struct Buf {
    __amdgpu_buffer_rsrc_t r;
    int pb;   // bytes per plane
};

__device__ __forceinline__ Buf make_buf(const float* base, int64_t floats, int64_t plane) {
    Buf b;
    b.r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0,
                                            (int)(floats * 4), 0x00020000);
    b.pb = (int)(plane * 4);
    return b;
}

// The view of species s of a lattice whose planes start at `lattice`.
template <int LAT>
__device__ __forceinline__ Buf species_buf(const float* lattice, int64_t plane, int s) {
    constexpr int Q = Lat<LAT>::Q;
    return make_buf(lattice + (int64_t)s * Q * plane, (int64_t)Q * plane, plane);
}

// Byte offset that lies beyond any species view (the host keeps every
// species below 2 GiB): a raw buffer load at it is range-checked and returns
// 0, which is exactly the contribution of a solid (beyond-the-wall) source.
constexpr unsigned kSolid = 0x80000000u;

// Sum of two byte offsets where either may carry kSolid.  Offsets are added as
// signed 32-bit values with saturation: an in-lattice offset plus a
// neighbour step stays exact, and a sum with kSolid in it stays at or below
// INT_MIN plus a few steps, out of range as an unsigned offset.  A plain add
// would let two markers (the node next to walls on two axes reading the
// corner source beyond both) cancel modulo 2^32 into an in-range read.
__device__ __forceinline__ unsigned oadd(unsigned a, unsigned b) {
    return (unsigned)__builtin_elementwise_add_sat((int)a, (int)b);
}

// value of plane p at byte offset `vb` (per lane)
__device__ __forceinline__ float ldb(const Buf& b, int p, unsigned vb) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)vb, p * b.pb, 0));
}
// Cache policy of the population stores (a launch writes every value once
// and reads none of them back).  kStoreNT, the non-temporal (`nt`) policy,
// suits states larger than the last-level cache; kStoreWT, device scope
// (`sc1`: written through to the last-level cache), suits states that fit in
// it and are read again from there by the next step.  Either changes no value
// and no coherence rule; the host picks one per context by the size of the
// two population buffers.
constexpr int kStoreNT = 2;
constexpr int kStoreWT = 16;
template <int POL = kStoreNT>
__device__ __forceinline__ void stb(const Buf& b, int p, unsigned vb, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.r, (int)vb,
                                          p * b.pb, POL);
}

// Neighbour index i+k on an axis of n nodes: wrapped when periodic, -1 when the
// source node is solid (beyond a wall).
__device__ __forceinline__ int nbr(int i, int k, int n, bool wall) {
    int j = i + k;
    if (j < 0) return wall ? -1 : j + n;
    if (j >= n) return wall ? -1 : j - n;
    return j;
}

// Weights of the source offsets -1, 0, +1 for a direction component of sign p
// of a species with triple L (given for Courant number +c).
struct W3 {
    float m, z, p;
};
__device__ __forceinline__ W3 wsel(int p, const float* L) {
    if (p > 0) return W3{L[0], L[1], L[2]};
    if (p < 0) return W3{L[2], L[1], L[0]};
    return W3{0.0f, 1.0f, 0.0f};
}

// Per-column geometry: byte offsets of the cross-section neighbours relative
// to the column (kSolid added for a solid neighbour), and whether they are
// solid.
struct Col {
    unsigned bxm, bxp, bym, byp;
    bool sxm, sxp, sym, syp;
};

// Cross-lane moves along a wave: lane i takes lane i-1's (from_left) or lane
// i+1's (from_right) value; the lane with no such neighbour takes `old`.
__device__ __forceinline__ float from_left(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_right(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
        __builtin_bit_cast(int, old), __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}

// How the gather reads a plane value and its x neighbours at a row.
// NbLoad: every value by its own load (any work-group shape).
struct NbLoad {
    static constexpr bool wave = false;
    __device__ __forceinline__ void trip(const Buf& b, int p, unsigned row, const Col& c,
                                         float& m, float& z, float& q) const {
        z = ldb(b, p, row);
        m = ldb(b, p, oadd(row, c.bxm));
        q = ldb(b, p, oadd(row, c.bxp));
    }
};

// NbWave: the 64 lanes of the wave hold the 64 consecutive columns of one row.
// A plane row is read once and the x neighbours are taken from the adjacent
// lanes; one more load, in which lane 0 reads the column before the row
// segment and lane 63 the one after it (the other lanes re-read their own
// value: the same cache line), supplies the two values beyond the wave's ends.
// Walls and periodicity enter through the same neighbour offsets as in
// NbLoad.  Called with every lane of the wave active.
struct NbWave {
    static constexpr bool wave = true;
    unsigned hx;   // per lane: bxm on lane 0, bxp on lane 63, 0 elsewhere
    __device__ __forceinline__ void trip(const Buf& b, int p, unsigned row, const Col&,
                                         float& m, float& z, float& q) const {
        z = ldb(b, p, row);
        const float h = ldb(b, p, oadd(row, hx));
        m = from_left(h, z);
        q = from_right(h, z);
    }
};

// x-pass of plane p around byte offset `row`.
template <int P0, class NB>
__device__ __forceinline__ float xpass(const Buf& b, int p, unsigned row, const Col& c, W3 w,
                                       const NB& nb) {
    if constexpr (P0 == 0) {
        return ldb(b, p, row);
    } else {
        float m, z, q;
        nb.trip(b, p, row, c, m, z, q);
        float v = w.z * z;
        v = fmaf(w.m, m, v);
        v = fmaf(w.p, q, v);
        return v;
    }
}

// Cross-section pass of one deviation plane around byte offset `cen`.
template <int LAT, int Q0, int Q1, class NB>
__device__ __forceinline__ float hpass(const Buf& b, int p, unsigned cen, const Col& c,
                                       const float* L, const NB& nb) {
    const W3 wx = wsel(Q0, L);
    if constexpr (Lat<LAT>::DIM == 2 || Q1 == 0) {
        return xpass<Q0>(b, p, cen, c, wx, nb);
    } else {
        const W3 wy = wsel(Q1, L);
        float v = wy.z * xpass<Q0>(b, p, cen, c, wx, nb);
        v = fmaf(wy.m, xpass<Q0>(b, p, oadd(cen, c.bym), c, wx, nb), v);
        v = fmaf(wy.p, xpass<Q0>(b, p, oadd(cen, c.byp), c, wx, nb), v);
        return v;
    }
}

// Reference stencil of one layer around the column (rest populations P0):
// the centre and the differences to the four cross-section neighbours (a
// solid neighbour, or a whole solid layer, reads as 0).
struct RhoLayer {
    float c, dxm, dxp, dym, dyp;
};

template <int LAT, class NB>
__device__ __forceinline__ RhoLayer rho_layer(const Buf& b, int p, unsigned cen, const Col& c,
                                              const NB& nb) {
    RhoLayer r;
    float m, q;
    nb.trip(b, p, cen, c, m, r.c, q);
    r.dxm = m - r.c;
    r.dxp = q - r.c;
    if constexpr (Lat<LAT>::DIM == 3) {
        r.dym = ldb(b, p, oadd(cen, c.bym)) - r.c;
        r.dyp = ldb(b, p, oadd(cen, c.byp)) - r.c;
    } else {
        r.dym = r.dyp = 0.0f;
    }
    return r;
}

// Per-lattice constants the gather needs, kept in scalar registers.
struct GatherConst {
    int nx, ny, nz, pitch, nm, walls, lstride;   // walls: wall mask; lstride: floats per layer
    float lam[MAXS][3];
};

__device__ __forceinline__ GatherConst gather_const(const LatParams& P, int dim) {
    GatherConst g;
    g.nx = P.nx; g.ny = P.ny; g.nz = P.nz; g.pitch = P.pitch;
    g.nm = dim == 2 ? P.ny : P.nz;
    g.walls = P.wall_mask;
    g.lstride = dim == 2 ? P.pitch : P.ny * P.pitch;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
        g.lam[s][0] = P.lam[s][0]; g.lam[s][1] = P.lam[s][1]; g.lam[s][2] = P.lam[s][2];
    }
    return g;
}

#define LBM_HP(CEN)                                                                      \
    ((Fr::p0(a) > 0)                                                                     \
         ? ((Fr::p1(a) > 0)   ? hpass<LAT, 1, 1>(B, pidx, CEN, col, L, nb)                    \
            : (Fr::p1(a) < 0) ? hpass<LAT, 1, -1>(B, pidx, CEN, col, L, nb)                   \
                              : hpass<LAT, 1, 0>(B, pidx, CEN, col, L, nb))                   \
     : (Fr::p0(a) < 0)                                                                   \
         ? ((Fr::p1(a) > 0)   ? hpass<LAT, -1, 1>(B, pidx, CEN, col, L, nb)                   \
            : (Fr::p1(a) < 0) ? hpass<LAT, -1, -1>(B, pidx, CEN, col, L, nb)                  \
                              : hpass<LAT, -1, 0>(B, pidx, CEN, col, L, nb))                  \
         : ((Fr::p1(a) > 0)   ? hpass<LAT, 0, 1>(B, pidx, CEN, col, L, nb)                    \
            : (Fr::p1(a) < 0) ? hpass<LAT, 0, -1>(B, pidx, CEN, col, L, nb)                   \
                              : hpass<LAT, 0, 0>(B, pidx, CEN, col, L, nb)))

// Per-column geometry of a gather (shared by the joint and per-species forms).
struct ColGeom {
    Col col;
    int sx, sy;            // wall side of the column (-1, 0, +1) on x / y
    unsigned colbase;      // byte offset of the column in layer 0
    unsigned lsb;          // bytes per layer
    bool wx, wy, wm;       // walls on x / y / the marching axis
};

template <int LAT>
__device__ __forceinline__ ColGeom col_geom(const GatherConst& G, int x, int y) {
    constexpr int DIM = Lat<LAT>::DIM;
    ColGeom g;
    g.wx = (G.walls & 1) != 0;
    g.wy = DIM == 3 && (G.walls & 2) != 0;
    g.wm = (G.walls & (1 << Frame<LAT>::MA)) != 0;
    const int xm = nbr(x, -1, G.nx, g.wx), xp = nbr(x, 1, G.nx, g.wx);
    g.col.sxm = xm < 0;
    g.col.sxp = xp < 0;
    g.col.bxm = xm < 0 ? kSolid : (unsigned)(xm - x) * 4u;
    g.col.bxp = xp < 0 ? kSolid : (unsigned)(xp - x) * 4u;
    g.col.bym = g.col.byp = 0u;
    g.col.sym = g.col.syp = false;
    if constexpr (DIM == 3) {
        const int ym = nbr(y, -1, G.ny, g.wy), yp = nbr(y, 1, G.ny, g.wy);
        g.col.sym = ym < 0;
        g.col.syp = yp < 0;
        g.col.bym = ym < 0 ? kSolid : (unsigned)((ym - y) * G.pitch) * 4u;
        g.col.byp = yp < 0 ? kSolid : (unsigned)((yp - y) * G.pitch) * 4u;
    }
    g.sx = g.wx ? (x == 0 ? -1 : (x == G.nx - 1 ? 1 : 0)) : 0;
    g.sy = g.wy ? (y == 0 ? -1 : (y == G.ny - 1 ? 1 : 0)) : 0;
    g.colbase = (unsigned)((DIM == 2 ? 0 : y * G.pitch) + x) * 4u;
    g.lsb = (unsigned)G.lstride * 4u;
    return g;
}

// byte offset of the column in layer ml (kSolid beyond a wall)
__device__ __forceinline__ unsigned layer_off(const ColGeom& g, int ml) {
    return ml < 0 ? oadd(kSolid, g.colbase) : (unsigned)ml * g.lsb + g.colbase;
}

// Species 1 (c = 1) at layer m: exact shift.  f_a(O) = f~_a(O - c_a), or
// f~_abar(O) when O - c_a is solid (halfway bounce-back); written without
// branches: a solid source reads the rest population at O itself (difference
// 0) and the plane of the opposite direction.  (Each shifted value is a single
// read here, so the cross-lane form would not save loads.)  With EQ (the
// equilibrium comparison boundary) a solid source contributes nothing here;
// eq_wall_terms adds what the solid node holds.
template <int LAT, bool EQ = false>
__device__ __forceinline__ void shift_layer(const Buf& B, const GatherConst& G, const ColGeom& g,
                                            int m, unsigned own, float& P0,
                                            float (&F)[Lat<LAT>::Q]) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    constexpr int DIM = La::DIM;
    const Col& col = g.col;
    const float r0 = ldb(B, 0, own);
    P0 = r0;
    F[0] = 0.0f;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        const int c0 = Fr::p0(a), c1 = Fr::p1(a), cm = Fr::pm(a);
        unsigned src = own;
        bool solid = false;
        if (c0 > 0) { src += col.bxm; solid = solid || col.sxm; }
        if (c0 < 0) { src += col.bxp; solid = solid || col.sxp; }
        if constexpr (DIM == 3) {
            if (c1 > 0) { src += col.bym; solid = solid || col.sym; }
            if (c1 < 0) { src += col.byp; solid = solid || col.syp; }
        }
        if (cm != 0) {
            const int ms = nbr(m, -cm, G.nm, g.wm);
            solid = solid || ms < 0;
            src += (unsigned)(ms - m) * g.lsb;
        }
        // the scalar offset names the lower of the two planes so that the
        // per-lane offset stays inside the buffer in both cases
        const int lo = a < La::opp(a) ? a : La::opp(a);
        const unsigned sp = solid ? own : src;
        const unsigned sg = solid ? own + (unsigned)((La::opp(a) - lo) * B.pb)
                                  : src + (unsigned)((a - lo) * B.pb);
        F[a] = fmaf(La::wr(a), ldb(B, 0, sp) - r0, ldb(B, lo, sg));
        if constexpr (EQ) {
            if (solid) F[a] = -La::wr(a) * r0;
        }
    }
}

// wall sides of the node at layer m along the lattice axes x, y, z (-1: next
// to the low wall, +1: next to the high wall, 0: not next to a wall)
struct Sides {
    int s[3];
    bool any;
};

// The equilibrium comparison boundary of Sec. 4.1 (the scheme the paper sets
// against Appendix A on the Loschmidt tube), for a node next to walls, added
// to a gather in which solid sources contributed nothing: a source node O + k
// beyond a wall holds the rest equilibrium w_a rho_s, rho_s the density of the
// fluid node it faces (O + k with each component that crosses a wall set to
// 0), and is interpolated over like any node (eq. Second_order_spatial_
// interpolation, the tensor product in 3-D), so f_a(O) gains
// w_a sum over solid k of Lambda_k(c_a) rho_s(k).  Densities from the stored
// form: rho = P0/w_0 + sum_{a>0} g_a.
template <int LAT>
__device__ __forceinline__ void eq_wall_terms(const Buf& B, const GatherConst& G, const ColGeom& g,
                                              int pb0, const float* L, unsigned own, int m,
                                              const Sides& sd, float (&F)[Lat<LAT>::Q]) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    constexpr int DIM = La::DIM;
    constexpr int K1 = DIM == 3 ? 1 : 0;
    const float iw0 = 1.0f / La::w(0);
    const int sx = sd.s[0], s1 = DIM == 3 ? sd.s[1] : 0, sm = sd.s[Fr::MA];
    auto pick = [](const W3& w, int k) { return k < 0 ? w.m : (k > 0 ? w.p : w.z); };
#pragma unroll
    for (int km = -1; km <= 1; ++km)
#pragma unroll
        for (int k1 = -K1; k1 <= K1; ++k1)
#pragma unroll
            for (int kx = -1; kx <= 1; ++kx) {
                const bool solx = kx != 0 && kx == sx;
                const bool sol1 = k1 != 0 && k1 == s1;
                const bool solm = km != 0 && km == sm;
                if (!(solx || sol1 || solm)) continue;
                // the facing fluid node: the in-lattice steps of k only
                unsigned cl = (km != 0 && !solm) ? layer_off(g, nbr(m, km, G.nm, g.wm)) : own;
                if (kx != 0 && !solx) cl += kx < 0 ? g.col.bxm : g.col.bxp;
                if (k1 != 0 && !sol1) cl += k1 < 0 ? g.col.bym : g.col.byp;
                float rho = ldb(B, pb0, cl) * iw0;
#pragma unroll
                for (int b = 1; b < Q; ++b) rho += ldb(B, pb0 + b, cl);
#pragma unroll
                for (int a = 1; a < Q; ++a) {
                    if ((Fr::p0(a) == 0 && kx != 0) || (Fr::p1(a) == 0 && k1 != 0) ||
                        (Fr::pm(a) == 0 && km != 0))
                        continue;
                    float wgt = pick(wsel(Fr::p0(a), L), kx) * pick(wsel(Fr::pm(a), L), km);
                    if constexpr (DIM == 3) wgt *= pick(wsel(Fr::p1(a), L), k1);
                    F[a] = fmaf(La::w(a) * wgt, rho, F[a]);
                }
            }
}

// Slot of direction a among the directions with a marching-axis component.
template <int LAT>
__host__ __device__ constexpr int mar_slot(int a) {
    int k = 0;
    for (int b = 1; b < a; ++b) k += Frame<LAT>::pm(b) != 0 ? 1 : 0;
    return k;
}
template <int LAT>
constexpr int kMarDirs = mar_slot<LAT>(Lat<LAT>::Q);

// The two marching-axis partial sums of every direction with a marching
// component (get/set(k, a): sum k of direction a), in registers.
template <int LAT, bool LDS = false>
struct MarchSums {
    float acc0[Lat<LAT>::Q], acc1[Lat<LAT>::Q];
    __device__ __forceinline__ float get(int k, int a) const { return k ? acc1[a] : acc0[a]; }
    __device__ __forceinline__ void set(int k, int a, float v) {
        if (k)
            acc1[a] = v;
        else
            acc0[a] = v;
    }
};
// The same sums in an LDS area of the wave's own ([2 kMarDirs][64] floats,
// each lane its column; no other lane reads them, so no barrier), so they
// hold no VGPRs.
template <int LAT>
struct MarchSums<LAT, true> {
    float* acc;   // this lane's element of slot 0
    __device__ __forceinline__ float get(int k, int a) const {
        return acc[(2 * mar_slot<LAT>(a) + k) * 64];
    }
    __device__ __forceinline__ void set(int k, int a, float v) {
        acc[(2 * mar_slot<LAT>(a) + k) * 64] = v;
    }
};

// Marching state of one heavier species: the marching-axis partial sums of
// its deviation planes and the reference stencil of layers m-1, m, m+1.
template <int LAT, bool LDS = false>
struct Heavy : MarchSums<LAT, LDS> {
    RhoLayer rl[3];
};

// Start the march of a heavier species (planes pb0 .. pb0+Q-1) at layer m0.
template <int LAT, class NB, bool HL>
__device__ __forceinline__ void heavy_begin(const Buf& B, const GatherConst& G, const ColGeom& g,
                                            int pb0, const float* L, int m0, Heavy<LAT, HL>& h,
                                            const NB& nb) {
    using Fr = Frame<LAT>;
    constexpr int Q = Lat<LAT>::Q;
    const Col& col = g.col;
    const int lm = nbr(m0, -1, G.nm, g.wm);
    const unsigned cm_ = layer_off(g, lm), c0_ = layer_off(g, m0);
    h.rl[0] = rho_layer<LAT>(B, pb0, cm_, col, nb);
    h.rl[1] = rho_layer<LAT>(B, pb0, c0_, col, nb);
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        if (Fr::pm(a) != 0) {
            const int pidx = pb0 + a;
            const W3 wmar = wsel(Fr::pm(a), L);
            const float hm = LBM_HP(cm_);
            const float h0 = LBM_HP(c0_);
            h.set(0, a, fmaf(wmar.z, h0, wmar.m * hm));
            h.set(1, a, wmar.m * h0);
        } else if constexpr (!HL) {
            h.set(0, a, 0.0f);
            h.set(1, a, 0.0f);
        }
    }
}

// One layer of a heavier species: second-order interpolation plus the
// impermeable-wall terms; side is the column's wall side on the wall axis.
template <int LAT, bool EQ = false, class NB, bool HL>
__device__ __forceinline__ void heavy_layer(const Buf& B, const GatherConst& G, const ColGeom& g,
                                            int pb0, const float* L, unsigned own, unsigned nxt,
                                            int m, const Sides& sd, Heavy<LAT, HL>& h, float& P0,
                                            float (&F)[Lat<LAT>::Q], const NB& nb) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    constexpr int DIM = La::DIM;
    const Col& col = g.col;
    h.rl[2] = rho_layer<LAT>(B, pb0, nxt, col, nb);
    const float rc = h.rl[1].c;
    P0 = rc;
    F[0] = 0.0f;
    // 3-D edge directions in the cross-section need the corner
    // x-differences of rows y-1 and y+1 of this layer
    float cxm[2] = {0.0f, 0.0f}, cxp[2] = {0.0f, 0.0f};
    if constexpr (DIM == 3) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const unsigned rr = oadd(own, j == 0 ? col.bym : col.byp);
            float cm, cc, cp;
            nb.trip(B, pb0, rr, col, cm, cc, cp);
            cxm[j] = cm - cc;
            cxp[j] = cp - cc;
        }
    }
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        const int pidx = pb0 + a;
        const W3 wxw = wsel(Fr::p0(a), L);
        const W3 wyw = wsel(Fr::p1(a), L);
        // reference part: delta_a = sum_k Lambda_k P0(O+k) - P0(O)
        auto xpart = [&](const RhoLayer& r) {
            return Fr::p0(a) != 0 ? fmaf(wxw.m, r.dxm, wxw.p * r.dxp) : 0.0f;
        };
        auto ypart = [&](const RhoLayer& r) {
            return Fr::p1(a) != 0 ? fmaf(wyw.m, r.dym, wyw.p * r.dyp) : 0.0f;
        };
        float delta;
        if (Fr::p0(a) != 0 && Fr::p1(a) != 0) {
            // 3-D xy edge: nested pass over rows y-1, y, y+1 of layer m
            const RhoLayer& r = h.rl[1];
            float v = wyw.z * xpart(r);
            v = fmaf(wyw.m, r.dym + fmaf(wxw.m, cxm[0], wxw.p * cxp[0]), v);
            v = fmaf(wyw.p, r.dyp + fmaf(wxw.m, cxm[1], wxw.p * cxp[1]), v);
            delta = v;
        } else if (Fr::pm(a) == 0) {
            delta = xpart(h.rl[1]) + ypart(h.rl[1]);
        } else {
            const W3 wmw = wsel(Fr::pm(a), L);
            // a solid layer reads as zeros: its term is -rc
            const RhoLayer& lo = h.rl[0];
            const RhoLayer& hi = h.rl[2];
            const float tlo = (lo.c - rc) + xpart(lo) + ypart(lo);
            const float thi = (hi.c - rc) + xpart(hi) + ypart(hi);
            const float tmid = xpart(h.rl[1]) + ypart(h.rl[1]);
            delta = fmaf(wmw.p, thi, fmaf(wmw.m, tlo, wmw.z * tmid));
        }
        // deviation part
        float Gv;
        if (Fr::pm(a) == 0) {
            Gv = LBM_HP(own);
        } else {
            const W3 wmar = wsel(Fr::pm(a), L);
            const float hn = LBM_HP(nxt);   // 0 beyond a wall
            const float a0 = h.get(0, a), a1 = h.get(1, a);
            Gv = fmaf(wmar.p, hn, a0);
            h.set(0, a, fmaf(wmar.z, hn, a1));
            h.set(1, a, wmar.m * hn);
        }
        F[a] = fmaf(La::wr(a), delta, Gv);
    }
    // impermeable walls (Appendix A): for a pointing away from the wall,
    // f_a(O) += lambda_+1(c) f~_a(O) + lambda_-1(c) f~_abar(O); with
    // f~ = (w/w_0) P0 + g and w_a = w_abar the reference part is
    // (w_a/w_0)(lambda_+1 + lambda_-1) P0(O).  Where walls meet, what the
    // node's populations would stream beyond the walls returns to the node,
    // split by the set of walls crossed: into the reversed direction if the
    // population moves toward one of them, else into its own direction.
    // For a direction pointing away from n_away of the node's walls and
    // toward n_tow of them that gives
    //   f_a += (1 - (1 - l+)^n_away) (1 - l-)^n_tow f~_a
    //        + (1 - (1 - l-)^n_away) f~_abar,
    // (l+- = lambda_+-1(c)), the Appendix A terms for a single wall.
    if constexpr (EQ) {
        if (sd.any) eq_wall_terms<LAT>(B, G, g, pb0, L, own, m, sd, F);
    } else if (sd.any) {
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            int na = 0, nt = 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const int p = sd.s[ax] * (ax == 0 ? La::cx(a) : (ax == 1 ? La::cy(a) : La::cz(a)));
                na += p < 0;
                nt += p > 0;
            }
            if (na == 0) continue;
            float c1 = L[2], c2 = L[0];
            if (na > 1 || nt > 0) {
                const float u0 = 1.0f - L[0], u2 = 1.0f - L[2];
                float p0a = u0, p2a = u2, p0t = 1.0f;
                for (int k = 1; k < na; ++k) {
                    p0a *= u0;
                    p2a *= u2;
                }
                for (int k = 0; k < nt; ++k) p0t *= u0;
                c1 = (1.0f - p2a) * p0t;
                c2 = 1.0f - p0a;
            }
            const float ga = ldb(B, pb0 + a, own);
            const float gb = ldb(B, pb0 + La::opp(a), own);
            F[a] += fmaf(c1, ga, c2 * gb) + La::wr(a) * (c1 + c2) * rc;
        }
    }
    h.rl[0] = h.rl[1];
    h.rl[1] = h.rl[2];
}

template <int LAT>
__device__ __forceinline__ Sides wall_sides(const GatherConst& G, const ColGeom& g, int m) {
    constexpr int DIM = Lat<LAT>::DIM;
    const int sm = g.wm ? (m == 0 ? -1 : (m == G.nm - 1 ? 1 : 0)) : 0;
    Sides r;
    r.s[0] = g.sx;
    r.s[1] = DIM == 2 ? sm : g.sy;
    r.s[2] = DIM == 3 ? sm : 0;
    r.any = (r.s[0] | r.s[1] | r.s[2]) != 0;
    return r;
}

// Forward pull gather of one column through layers [m0, m1), all species
// (B: the species views); calls op(P0, F, m, own) for every layer m (own:
// byte offset of the node within a plane).
template <int LAT, int NS, bool EQ = false, class Op>
__device__ __forceinline__ void march(const Buf (&B)[NS], const GatherConst& G, int x, int y,
                                      int m0, int m1, Op& op) {
    constexpr int Q = Lat<LAT>::Q;
    const ColGeom g = col_geom<LAT>(G, x, y);
    const NbLoad nb{};
    Heavy<LAT> h[NS > 1 ? NS - 1 : 1];
#pragma unroll
    for (int s = 1; s < NS; ++s) heavy_begin<LAT>(B[s], G, g, 0, G.lam[s], m0, h[s - 1], nb);
    for (int m = m0; m < m1; ++m) {
        const int mp = nbr(m, 1, G.nm, g.wm);
        const unsigned own = layer_off(g, m);
        const unsigned nxt = layer_off(g, mp);
        const Sides sd = wall_sides<LAT>(G, g, m);
        float P0[NS], F[NS][Q];
        shift_layer<LAT, EQ>(B[0], G, g, m, own, P0[0], F[0]);
        if constexpr (EQ) {
            if (sd.any) eq_wall_terms<LAT>(B[0], G, g, 0, G.lam[0], own, m, sd, F[0]);
        }
#pragma unroll
        for (int s = 1; s < NS; ++s)
            heavy_layer<LAT, EQ>(B[s], G, g, 0, G.lam[s], own, nxt, m, sd, h[s - 1], P0[s], F[s],
                                 nb);
        op(P0, F, m, own);
    }
}

template <int LAT, bool HL, class NB, class Op>
__device__ __forceinline__ void march1_nb(const Buf& B, const GatherConst& G, int s,
                                          const float (&L)[3], const ColGeom& g, int m0, int m1,
                                          Op& op, const NB& nb, float* macc) {
    constexpr int Q = Lat<LAT>::Q;
    Heavy<LAT, HL> h;
    if constexpr (HL) h.acc = macc;
    if (s > 0) heavy_begin<LAT>(B, G, g, 0, L, m0, h, nb);
    for (int m = m0; m < m1; ++m) {
        const int mp = nbr(m, 1, G.nm, g.wm);
        const unsigned own = layer_off(g, m);
        const unsigned nxt = layer_off(g, mp);
        float P0, F[Q];
        if (s == 0)
            shift_layer<LAT>(B, G, g, m, own, P0, F);
        else
            heavy_layer<LAT>(B, G, g, 0, L, own, nxt, m, wall_sides<LAT>(G, g, m), h, P0, F,
                             nb);
        op(P0, F, m, own);
    }
}

// The same gather for one species s (uniform over the wave; B its view) with
// weight triple L; calls op(P0, F, m, own) with the species' values.  With wave_row
// the wave's 64 lanes are 64 consecutive columns of one row (in order) and the
// x neighbours are taken across lanes.  lane_zero marks a lane whose reads
// all return 0.  With HL the marching partial sums live in the LDS area
// macc (this lane's element of the wave's [2 kMarDirs][64] floats).
template <int LAT, class Op, bool HL = false>
__device__ __forceinline__ void march1(const Buf& B, const GatherConst& G, int s,
                                       const float (&L)[3], int x, int y, bool lane_zero,
                                       bool wave_row, int m0, int m1, Op& op,
                                       float* macc = nullptr) {
    ColGeom g = col_geom<LAT>(G, x, y);
    if (lane_zero) g.colbase += kSolid;
    if (wave_row) {
        const unsigned lane = __lane_id();
        NbWave nb{lane == 0 ? g.col.bxm : (lane == 63 ? g.col.bxp : 0u)};
        march1_nb<LAT, HL>(B, G, s, L, g, m0, m1, op, nb, macc);
    } else {
        march1_nb<LAT, HL>(B, G, s, L, g, m0, m1, op, NbLoad{}, macc);
    }
}

// Column of lane `lane` of a tile of 64 columns: x fastest over bx columns,
// then y (3-D).  Returns whether the lane lies in the lattice; a lane beyond
// it stores nothing and follows the column after the row's last one (the
// wrapped column when x is periodic, a lane whose reads return 0 at an x
// wall: `zero`), and in y the last row.  The last column's right neighbour in
// the cross-lane gather is then the right value.
template <int LAT>
__device__ __forceinline__ bool tile_column(const Tile& T, const LatParams& P, int lane, int bx,
                                            int& x, int& y, bool& zero) {
    constexpr int DIM = Lat<LAT>::DIM;
    x = T.x0 + (DIM == 3 ? lane % bx : lane);
    y = DIM == 3 ? T.y0 + lane / bx : 0;
    const bool inside = x < P.nx && (DIM == 2 || y < P.ny);
    zero = false;
    if (x >= P.nx) {
        if (P.wall_mask & 1) {
            x = P.nx - 1;
            zero = true;
        } else {
            x %= P.nx;
        }
    }
    if (DIM == 3 && y >= P.ny) y = P.ny - 1;
    return inside;
}

// tile_column for a work-group of W segments of 64 columns (W = bx by / 64):
// with W = 1 the lanes are laid out as tile_column; with W > 1 (bx a multiple
// of 64) segment seg is the 64 columns starting at x0 + 64 (seg mod (bx/64))
// in row y0 + seg / (bx/64), lane = column.
template <int LAT>
__device__ __forceinline__ bool tile_column_seg(const Tile& T, const LatParams& P, int lane, int bx,
                                                int seg, int W, int& x, int& y, bool& zero) {
    if (W == 1) return tile_column<LAT>(T, P, lane, bx, x, y, zero);
    const int per_row = bx >> 6;
    Tile S = T;
    S.x0 = T.x0 + 64 * (seg % per_row);
    S.y0 = T.y0 + seg / per_row;
    return tile_column<LAT>(S, P, lane, 64, x, y, zero);
}

#undef LBM_HP

}  // namespace lbmmc
