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
// read neighbouring columns straight from global memory (L1/L2 hits: the
// neighbouring lanes of the same instruction read the same rows), and the
// pass along the marching axis is carried in registers (two running partial
// sums per deviation plane, three layers of the density stencil), so every
// value of a layer is fetched from HBM about once.  Species 1 (c = 1) is an
// exact one-node shift.
//
// For every node the gather hands over, per species s:
//   P0[s]     the stored rest population at the node (it does not stream),
//   F[s][a]   f_a(O) - w_a r*(O) for a >= 1, f_a the streamed population
//             (for a = 0 this is zero).
// With the FP32 weight triples summing to exactly 1 and the wall terms handing
// back the stored weights that a solid layer would have received (Appendix A),
// the update moves mass without systematic drift.
#pragma once

#include "common.hpp"
#include "lattice.hpp"

namespace lbmmc {

// Neighbour index i+k on an axis of n nodes: wrapped when periodic, -1 when the
// source node is solid (beyond a wall).
__device__ __forceinline__ int nbr(int i, int k, int n, bool wall) {
    int j = i + k;
    if (j < 0) return wall ? -1 : j + n;
    if (j >= n) return wall ? -1 : j - n;
    return j;
}

// Weights of the source offsets -1, 0, +1 for a direction component of sign P
// of a species with triple L (given for Courant number +c).
struct W3 {
    float m, z, p;
};
template <int P>
__device__ __forceinline__ W3 wsel(const float* L) {
    if constexpr (P > 0) return W3{L[0], L[1], L[2]};
    else if constexpr (P < 0) return W3{L[2], L[1], L[0]};
    else return W3{0.0f, 1.0f, 0.0f};
}
__device__ __forceinline__ W3 wsel_rt(int p, const float* L) {
    if (p > 0) return W3{L[0], L[1], L[2]};
    if (p < 0) return W3{L[2], L[1], L[0]};
    return W3{0.0f, 1.0f, 0.0f};
}

template <int P0>
__device__ __forceinline__ float xpass(const float* __restrict__ row, int x, int xm, int xp, W3 w) {
    if constexpr (P0 == 0) {
        return row[x];
    } else {
        float v = w.z * row[x];
        if (xm >= 0) v = fmaf(w.m, row[xm], v);
        if (xp >= 0) v = fmaf(w.p, row[xp], v);
        return v;
    }
}

// Cross-section pass of one deviation plane at layer ml (a valid layer).
template <int LAT, int Q0, int Q1>
__device__ __forceinline__ float hpass(const float* __restrict__ pl, int pitch, int ny, int ml,
                                       int x, int xm, int xp, int y, int ym, int yp,
                                       const float* L) {
    const W3 wx = wsel<Q0>(L);
    if constexpr (Lat<LAT>::DIM == 2) {
        return xpass<Q0>(pl + (int64_t)ml * pitch, x, xm, xp, wx);
    } else {
        const float* lay = pl + (int64_t)ml * ny * pitch;
        if constexpr (Q1 == 0) {
            return xpass<Q0>(lay + (int64_t)y * pitch, x, xm, xp, wx);
        } else {
            const W3 wy = wsel<Q1>(L);
            float v = wy.z * xpass<Q0>(lay + (int64_t)y * pitch, x, xm, xp, wx);
            if (ym >= 0) v = fmaf(wy.m, xpass<Q0>(lay + (int64_t)ym * pitch, x, xm, xp, wx), v);
            if (yp >= 0) v = fmaf(wy.p, xpass<Q0>(lay + (int64_t)yp * pitch, x, xm, xp, wx), v);
            return v;
        }
    }
}

template <int LAT>
__device__ __forceinline__ int64_t node_off(int pitch, int ny, int x, int y, int m) {
    if constexpr (Lat<LAT>::DIM == 2) return (int64_t)m * pitch + x;
    else return ((int64_t)m * ny + y) * pitch + x;
}

// Reference stencil of one layer around the column (rest populations P0):
// the centre and the differences to the four cross-section neighbours (a
// solid neighbour counts as 0).  `ok` is false for a solid layer beyond a wall.
struct RhoLayer {
    float c, dxm, dxp, dym, dyp;
    bool ok;
};

template <int LAT>
__device__ __forceinline__ RhoLayer rho_layer(const float* __restrict__ rp, int pitch, int ny,
                                              int ml, int x, int xm, int xp, int y, int ym,
                                              int yp) {
    RhoLayer r;
    if (ml < 0) {
        r.c = r.dxm = r.dxp = r.dym = r.dyp = 0.0f;
        r.ok = false;
        return r;
    }
    r.ok = true;
    if constexpr (Lat<LAT>::DIM == 2) {
        const float* row = rp + (int64_t)ml * pitch;
        r.c = row[x];
        r.dxm = (xm >= 0 ? row[xm] : 0.0f) - r.c;
        r.dxp = (xp >= 0 ? row[xp] : 0.0f) - r.c;
        r.dym = r.dyp = 0.0f;
    } else {
        const float* lay = rp + (int64_t)ml * ny * pitch;
        const float* row = lay + (int64_t)y * pitch;
        r.c = row[x];
        r.dxm = (xm >= 0 ? row[xm] : 0.0f) - r.c;
        r.dxp = (xp >= 0 ? row[xp] : 0.0f) - r.c;
        r.dym = (ym >= 0 ? lay[(int64_t)ym * pitch + x] : 0.0f) - r.c;
        r.dyp = (yp >= 0 ? lay[(int64_t)yp * pitch + x] : 0.0f) - r.c;
    }
    return r;
}

// Copy of the per-lattice constants the gather needs, kept in scalar registers.
struct GatherConst {
    int nx, ny, nz, pitch, nm, wall_axis;
    int64_t plane;
    float lam[MAXS][3];
};

__device__ __forceinline__ GatherConst gather_const(const LatParams& P, int dim) {
    GatherConst g;
    g.nx = P.nx; g.ny = P.ny; g.nz = P.nz; g.pitch = P.pitch;
    g.nm = dim == 2 ? P.ny : P.nz;
    g.wall_axis = P.wall_axis;
    g.plane = P.plane;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
        g.lam[s][0] = P.lam[s][0]; g.lam[s][1] = P.lam[s][1]; g.lam[s][2] = P.lam[s][2];
    }
    return g;
}

#define LBM_HP(ML)                                                                                \
    ((Fr::p0(a) > 0)                                                                              \
         ? ((Fr::p1(a) > 0)   ? hpass<LAT, 1, 1>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L)  \
            : (Fr::p1(a) < 0) ? hpass<LAT, 1, -1>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L) \
                              : hpass<LAT, 1, 0>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L)) \
     : (Fr::p0(a) < 0)                                                                            \
         ? ((Fr::p1(a) > 0)   ? hpass<LAT, -1, 1>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L) \
            : (Fr::p1(a) < 0) ? hpass<LAT, -1, -1>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L) \
                              : hpass<LAT, -1, 0>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L)) \
         : ((Fr::p1(a) > 0)   ? hpass<LAT, 0, 1>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L)  \
            : (Fr::p1(a) < 0) ? hpass<LAT, 0, -1>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L) \
                              : hpass<LAT, 0, 0>(pl, G.pitch, G.ny, ML, x, xm, xp, y, ym, yp, L)))

// Forward pull gather of one column through layers [m0, m1); calls
// op(P0, F, m, own) for every layer m.
template <int LAT, int NS, class Op>
__device__ __forceinline__ void march(const float* __restrict__ lb, const GatherConst& G, int x,
                                      int y, int m0, int m1, Op& op) {
    using Fr = Frame<LAT>;
    using La = Lat<LAT>;
    constexpr int Q = La::Q;
    constexpr int DIM = La::DIM;
    const bool wx = G.wall_axis == 0;
    const bool wy = DIM == 3 && G.wall_axis == 1;
    const bool wm = G.wall_axis == Fr::MA;
    const int xm = nbr(x, -1, G.nx, wx), xp = nbr(x, 1, G.nx, wx);
    int ym = 0, yp = 0;
    if constexpr (DIM == 3) {
        ym = nbr(y, -1, G.ny, wy);
        yp = nbr(y, 1, G.ny, wy);
    }
    const int sx = wx ? (x == 0 ? -1 : (x == G.nx - 1 ? 1 : 0)) : 0;
    const int sy = wy ? (y == 0 ? -1 : (y == G.ny - 1 ? 1 : 0)) : 0;

    // marching-axis partial sums of the deviation planes, and the density
    // stencil of layers m-1, m, m+1 (heavier species only)
    float acc0[NS][Q], acc1[NS][Q];
    RhoLayer rl[NS][3];
    {
        const int lm = nbr(m0, -1, G.nm, wm);
#pragma unroll
        for (int s = 1; s < NS; ++s) {
            const float* rp = lb + (int64_t)(s * Q) * G.plane;
            rl[s][0] = rho_layer<LAT>(rp, G.pitch, G.ny, lm, x, xm, xp, y, ym, yp);
            rl[s][1] = rho_layer<LAT>(rp, G.pitch, G.ny, m0, x, xm, xp, y, ym, yp);
            const float* L = G.lam[s];
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                if (Fr::pm(a) != 0) {
                    const float* pl = lb + (int64_t)(s * Q + a) * G.plane;
                    const W3 wmar = wsel_rt(Fr::pm(a), L);
                    float hm = 0.0f;
                    if (lm >= 0) hm = LBM_HP(lm);
                    const float h0 = LBM_HP(m0);
                    acc0[s][a] = fmaf(wmar.z, h0, wmar.m * hm);
                    acc1[s][a] = wmar.m * h0;
                } else {
                    acc0[s][a] = 0.0f;
                    acc1[s][a] = 0.0f;
                }
            }
        }
    }

    for (int m = m0; m < m1; ++m) {
        const int mp = nbr(m, 1, G.nm, wm);
        const int sm = wm ? (m == 0 ? -1 : (m == G.nm - 1 ? 1 : 0)) : 0;
        const int64_t own = node_off<LAT>(G.pitch, G.ny, x, y, m);
        float P0[NS], F[NS][Q];
        // ------------------------------------------------ species 1: exact shift
        {
            const float r0 = lb[own];
            P0[0] = r0;
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const float* pl = lb + (int64_t)a * G.plane;
                const int c0 = Fr::p0(a), c1 = Fr::p1(a), cm = Fr::pm(a);
                int xs = x, ys = y, ms = m;
                bool solid = false;
                if (c0 > 0) xs = xm; else if (c0 < 0) xs = xp;
                if (c0 != 0 && xs < 0) solid = true;
                if constexpr (DIM == 3) {
                    if (c1 > 0) ys = ym; else if (c1 < 0) ys = yp;
                    if (c1 != 0 && ys < 0) solid = true;
                }
                if (cm != 0) {
                    ms = nbr(m, -cm, G.nm, wm);
                    if (ms < 0) solid = true;
                }
                if (!solid) {
                    const int64_t src = node_off<LAT>(G.pitch, G.ny, xs, ys, ms);
                    F[0][a] = fmaf(La::wr(a), lb[src] - r0, pl[src]);
                } else {
                    // halfway bounce-back: f_a(O) = f~_abar(O)
                    F[0][a] = lb[(int64_t)La::opp(a) * G.plane + own];
                }
            }
        }
        // -------------------------------- heavier species: second-order interpolation
#pragma unroll
        for (int s = 1; s < NS; ++s) {
            const float* L = G.lam[s];
            const float* rp = lb + (int64_t)(s * Q) * G.plane;
            rl[s][2] = rho_layer<LAT>(rp, G.pitch, G.ny, mp, x, xm, xp, y, ym, yp);
            const float rc = rl[s][1].c;
            P0[s] = rc;
            // 3-D edge directions in the cross-section need the corner
            // x-differences of rows y-1 and y+1 of this layer
            float cxm[2] = {0.0f, 0.0f}, cxp[2] = {0.0f, 0.0f};
            if constexpr (DIM == 3) {
                const float* lay = rp + (int64_t)m * G.ny * G.pitch;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int yy = j == 0 ? ym : yp;
                    if (yy >= 0) {
                        const float* row = lay + (int64_t)yy * G.pitch;
                        const float cc = row[x];
                        cxm[j] = (xm >= 0 ? row[xm] : 0.0f) - cc;
                        cxp[j] = (xp >= 0 ? row[xp] : 0.0f) - cc;
                    }
                }
            }
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                const float* pl = lb + (int64_t)(s * Q + a) * G.plane;
                const W3 wxw = wsel_rt(Fr::p0(a), L);
                const W3 wyw = wsel_rt(Fr::p1(a), L);
                // reference part: delta_a = sum_k Lambda_k P0(O+k) - P0(O)
                float delta;
                auto xpart = [&](const RhoLayer& r) {
                    return Fr::p0(a) != 0 ? fmaf(wxw.m, r.dxm, wxw.p * r.dxp) : 0.0f;
                };
                auto ypart = [&](const RhoLayer& r) {
                    return Fr::p1(a) != 0 ? fmaf(wyw.m, r.dym, wyw.p * r.dyp) : 0.0f;
                };
                if (Fr::p0(a) != 0 && Fr::p1(a) != 0) {
                    // 3-D xy edge: nested pass over rows y-1, y, y+1 of layer m
                    const RhoLayer& r = rl[s][1];
                    float v = wyw.z * xpart(r);
                    if (ym >= 0) v = fmaf(wyw.m, r.dym + fmaf(wxw.m, cxm[0], wxw.p * cxp[0]), v);
                    else v = fmaf(wyw.m, r.dym, v);
                    if (yp >= 0) v = fmaf(wyw.p, r.dyp + fmaf(wxw.m, cxm[1], wxw.p * cxp[1]), v);
                    else v = fmaf(wyw.p, r.dyp, v);
                    delta = v;
                } else if (Fr::pm(a) == 0) {
                    delta = xpart(rl[s][1]) + ypart(rl[s][1]);
                } else {
                    const W3 wmw = wsel_rt(Fr::pm(a), L);
                    const RhoLayer& lo = rl[s][0];
                    const RhoLayer& hi = rl[s][2];
                    const float tlo = lo.ok ? (lo.c - rc) + xpart(lo) + ypart(lo) : -rc;
                    const float thi = hi.ok ? (hi.c - rc) + xpart(hi) + ypart(hi) : -rc;
                    const float tmid = xpart(rl[s][1]) + ypart(rl[s][1]);
                    delta = fmaf(wmw.p, thi, fmaf(wmw.m, tlo, wmw.z * tmid));
                }
                // deviation part
                float Gv;
                if (Fr::pm(a) == 0) {
                    Gv = LBM_HP(m);
                } else {
                    const W3 wmar = wsel_rt(Fr::pm(a), L);
                    float hn = 0.0f;
                    if (mp >= 0) hn = LBM_HP(mp);
                    Gv = fmaf(wmar.p, hn, acc0[s][a]);
                    acc0[s][a] = fmaf(wmar.z, hn, acc1[s][a]);
                    acc1[s][a] = wmar.m * hn;
                }
                F[s][a] = fmaf(La::wr(a), delta, Gv);
            }
            // impermeable walls (Appendix A): for a pointing away from the wall,
            // f_a(O) += lambda_+1(c) f~_a(O) + lambda_-1(c) f~_abar(O); with
            // f~ = (w/w_0) P0 + g and w_a = w_abar the reference part is
            // (w_a/w_0)(lambda_+1 + lambda_-1) P0(O).
            const int axis = G.wall_axis;
            const int side = axis == 0 ? sx : (axis == Fr::MA ? sm : sy);
            if (side != 0) {
#pragma unroll
                for (int a = 1; a < Q; ++a) {
                    const int ca = Fr::comp(a, axis);
                    if (side * ca < 0) {
                        const float ga = lb[(int64_t)(s * Q + a) * G.plane + own];
                        const float gb = lb[(int64_t)(s * Q + La::opp(a)) * G.plane + own];
                        F[s][a] += fmaf(L[2], ga, L[0] * gb) + La::wr(a) * (L[2] + L[0]) * rc;
                    }
                }
            }
            rl[s][0] = rl[s][1];
            rl[s][1] = rl[s][2];
        }
        op(P0, F, m, own);
    }
}

#undef LBM_HP

}  // namespace lbmmc
