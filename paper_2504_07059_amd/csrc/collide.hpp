// Per-node collision with forcing, in registers (FP32), in deviation form.
//
// Input per species (from the gather): P0 (the stored rest population at the
// node, reference density r* = P0/w_0) and F_a = f_a - w_a r* (a >= 1).  Then
//   rho_i  = r* + sum_{a>=1} F_a                          eq. (zeroth_order_moment)
//   rho_i u_i^eq = sum_a e f + F_i/2 = c_i sum_a c_a F_a + rho_i g/2
//                                                     eq. (first_order_moment_force)
//            (a species with rho_i below 1e-30 takes u_i^eq = g/2)
//   rho = sum rho_i, u = sum w_i u_i^eq                   eqs. (Sirovich_mixture_*)
//   n = sum rho_i/M_i, p = n M_1 c_{s,1}^2                (Sec. 3, Sec. 4.1)
//   1/tau_ij from eq. (relation_tauij_diff_coeff)         (tau_solve)
//   f~ = f - (f - f^(0))/tau_i + sum_j Omega^ij + (1 - 1/(2 tau_i)) S
//        with f^(eq), f^(0) of eq. (feqi0), Omega^ij of eq.
//        (Cross_collision_Sirovich), S of eq. (CE_forcing_term_discretized),
//        plus (forcing 1) the diffusion-driven contribution S_diff of eq.
//        (improved_forcing_scheme) with Theta_i of eq. (CE_theta_definition),
//        or (forcing 2) that whole equation, - S_p + S_rho + S_diff, with
//        the density gradients of field_grad;
// everything is evaluated as a deviation from w_a rho_i (collision conserves
// rho_i).  The result is stored as P0' = f~_0 and g_a = f~_a - (w_a/w_0) P0'
// (a >= 1); the rounding error of P0' is handed to the g_a in proportion to
// w_a, so the stored state keeps rho_i to the precision of the deviations.
#pragma once

#include "common.hpp"
#include "lattice.hpp"

namespace lbmmc {

struct CollConst {
    float c[MAXS], inv_cs2[MAXS], inv_tau[MAXS], fpref[MAXS], invM[MAXS], kdiff[MAXS], cs2[MAXS];
    float K[MAXS][MAXS];
    float g[3];
};

__device__ __forceinline__ CollConst coll_const(const LatParams& P) {
    CollConst C;
#pragma unroll
    for (int s = 0; s < MAXS; ++s) {
        C.c[s] = P.c[s]; C.inv_cs2[s] = P.inv_cs2[s]; C.inv_tau[s] = P.inv_tau[s];
        C.fpref[s] = P.fpref[s]; C.invM[s] = P.invM[s]; C.kdiff[s] = P.kdiff[s];
        C.cs2[s] = P.cs2[s];
#pragma unroll
        for (int t = 0; t < MAXS; ++t) C.K[s][t] = P.K[s][t];
    }
    C.g[0] = P.g[0]; C.g[1] = P.g[1]; C.g[2] = P.g[2];
    return C;
}

// integer direction dotted with a vector (exact adds)
template <int LAT>
__device__ __forceinline__ float cdot(int a, float vx, float vy, float vz) {
    using L = Lat<LAT>;
    float r = 0.0f;
    if (L::cx(a) == 1) r += vx; else if (L::cx(a) == -1) r -= vx;
    if (L::cy(a) == 1) r += vy; else if (L::cy(a) == -1) r -= vy;
    if (L::DIM == 3) {
        if (L::cz(a) == 1) r += vz; else if (L::cz(a) == -1) r -= vz;
    }
    return r;
}

// 1/x as the hardware reciprocal refined by one Newton step (about 1 ulp;
// x is a positive, normal density-like quantity wherever this is used).
__device__ __forceinline__ float rcp_nr(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Cross-relaxation solve.  For the pairs (i, j), i < j, that share the larger
// index j, eq. (relation_tauij_diff_coeff) with the index convention of the
// ternary solution of Sec. 4.1 reads (D + d rho^T) y = R_j d with
//   D_i = rho_j/D_ij + 2 n^2 M_i M_j/p,  d_i = 1/D_ij,
//   R_j = 2 rho - sum_{s>j} rho_s y_js  (known once columns s > j are done),
// a diagonal matrix plus a rank-one term, whose solution is
//   y_ij = R_j / (E_ij (1 + q_j)),  E_ij = rho_j + n K_ij,  q_j = sum_{i<j} rho_i/E_ij,
// with K_ij = 2 M_i M_j D_ij/(M_1 c_{s,1}^2) = 6 M_i M_j D_ij (dt = 1).  All
// E_ij > 0, so no pivoting is needed.
template <int NS>
__device__ __forceinline__ void tau_solve(const float (&rho)[NS], float R, float n,
                                          const CollConst& C, float (&y)[NS][NS]) {
#pragma unroll
    for (int j = NS - 1; j >= 1; --j) {
        float Rj = 2.0f * R;
#pragma unroll
        for (int s = j + 1; s < NS; ++s) Rj -= rho[s] * y[j][s];
        float iE[NS];
        float q = 0.0f;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            iE[i] = rcp_nr(fmaf(n, C.K[i][j], rho[j]));
            q += rho[i] * iE[i];
        }
        const float t = Rj * rcp_nr(1.0f + q);
#pragma unroll
        for (int i = 0; i < j; ++i) {
            y[i][j] = t * iE[i];
            y[j][i] = y[i][j];
        }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) y[i][i] = 0.0f;
}

constexpr float kRhoTiny = 1e-30f;

// Density, force-shifted equilibrium velocity and the deviation-form input of
// one species at one node (c: the species' speed).
template <int LAT>
__device__ __forceinline__ void species_moments(float P0, const float (&F)[Lat<LAT>::Q], float c,
                                                const float (&g)[3], float& rho, float& dlt,
                                                float (&ue)[3]) {
    constexpr int Q = Lat<LAT>::Q;
    using L = Lat<LAT>;
    float sf = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        const float v = F[a];
        sf += v;
        if (L::cx(a) == 1) jx += v; else if (L::cx(a) == -1) jx -= v;
        if (L::cy(a) == 1) jy += v; else if (L::cy(a) == -1) jy -= v;
        if (L::cz(a) == 1) jz += v; else if (L::cz(a) == -1) jz -= v;
    }
    dlt = sf;
    const float r = fmaf(P0, L::inv_w0, sf);
    rho = r;
    if (fabsf(r) > kRhoTiny) {
        const float cr = c * rcp_nr(r);
        ue[0] = fmaf(jx, cr, 0.5f * g[0]);
        ue[1] = fmaf(jy, cr, 0.5f * g[1]);
        ue[2] = fmaf(jz, cr, 0.5f * g[2]);
    } else {
        ue[0] = 0.5f * g[0];
        ue[1] = 0.5f * g[1];
        ue[2] = 0.5f * g[2];
    }
}

// Store transform: from the deviations gt_a = f~_a - w_a rho (a >= 1) with
// rho = P0/w_0 + dlt, produce P0' = f~_0 rounded to float and
// g_a = f~_a - (w_a/w_0) P0' + w_a (f~_0 - P0')/(1 - w_0).  With
// T = f~_0 - P0 = w_0 dlt - sum gt and d0 = P0 - P0' (exact: P0' is close to
// P0), g_a = gt_a + w_a e with e = d0/w_0 + dlt + (d0 + T)/(1 - w_0); all
// small numbers.  In exact arithmetic P0'/w_0 + sum_{a>=1} g_a = rho.
template <int LAT>
__device__ __forceinline__ float store_transform(float P0, float dlt, float sgt, float& e) {
    using L = Lat<LAT>;
    const float T = fmaf(L::w(0), dlt, -sgt);
    const float P0n = P0 + T;
    const float d0 = P0 - P0n;
    e = fmaf(d0, L::inv_w0, dlt) + (d0 + T) * L::inv_1mw0;
    return P0n;
}

// Mixture quantities of one node: rho, n, 1/rho, u and u.u.
struct Mix {
    float R, n, iR, U[3], uu;
};

template <int NS>
__device__ __forceinline__ Mix mixture(const float (&rho)[NS], const float (&ue)[NS][3],
                                       const CollConst& C) {
    Mix x;
    x.R = 0.0f;
    x.n = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        x.R += rho[s];
        x.n = fmaf(rho[s], C.invM[s], x.n);
    }
    x.iR = rcp_nr(x.R);
#pragma unroll
    for (int d = 0; d < 3; ++d) x.U[d] = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) x.U[d] = fmaf(rho[s], ue[s][d], x.U[d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) x.U[d] *= x.iR;
    x.uu = x.U[0] * x.U[0] + x.U[1] * x.U[1] + x.U[2] * x.U[2];
    return x;
}

// friction vector of species i: V_i = sum_j (rho_j y_ij / rho)(u_i^eq - u_j^eq)
template <int NS>
__device__ __forceinline__ void friction(int i, const float (&rho)[NS], const float (&ue)[NS][3],
                                         const float (&y)[NS][NS], float iR, float (&V)[3]) {
    V[0] = V[1] = V[2] = 0.0f;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if (j == i) continue;
        const float wij = rho[j] * y[i][j] * iR;
#pragma unroll
        for (int d = 0; d < 3; ++d) V[d] = fmaf(wij, ue[i][d] - ue[j][d], V[d]);
    }
}

// Per-species constants of one species (kd = 1/(2 tau - 1), used with FRC >= 1;
// cs2 = c_s^2, used with FRC 2).
struct SpeciesConst {
    float c, ics, itau, fp, kd, cs2;
};

// Density gradients at a node (FRC 2): of the species' own density and of
// the mixture density.
struct Grads {
    float gi[3], gm[3];
};

// Derivative along one axis of a node field, at index i of n nodes (reading
// of the paper's silent discretisation): (phi(i+1) - phi(i-1))/2, wrapped on
// a periodic axis; on a wall axis (n >= 3) the first and last nodes take the
// one-sided second-order differences (-3 phi_0 + 4 phi_1 - phi_2)/2 and
// (3 phi_{n-1} - 4 phi_{n-2} + phi_{n-3})/2.  at(j) reads the field at index j.
template <class At>
__device__ __forceinline__ float axis_diff(At at, int i, int n, bool wall) {
    if (wall) {
        if (i == 0) return 0.5f * (fmaf(4.0f, at(1), -3.0f * at(0)) - at(2));
        if (i == n - 1) return 0.5f * (fmaf(3.0f, at(n - 1), at(n - 3)) - 4.0f * at(n - 2));
        return 0.5f * (at(i + 1) - at(i - 1));
    }
    const int ip = i + 1 == n ? 0 : i + 1, im = i == 0 ? n - 1 : i - 1;
    return 0.5f * (at(ip) - at(im));
}

// Gradient of a dense node field (node index (z ny + y) nx + x) at (x, y, z)
// of a lattice with the given shape and wall mask (bit a: walls on axis a).
template <int DIM, class Phi>
__device__ __forceinline__ void field_grad(Phi phi, int nx, int ny, int nz, int wall_mask, int x,
                                           int y, int z, float (&g)[3]) {
    g[0] = axis_diff([&](int j) { return phi(((int64_t)z * ny + y) * nx + j); }, x, nx,
                     (wall_mask & 1) != 0);
    g[1] = axis_diff([&](int j) { return phi(((int64_t)z * ny + j) * nx + x); }, y, ny,
                     (wall_mask & 2) != 0);
    g[2] = DIM == 3 ? axis_diff([&](int j) { return phi(((int64_t)j * ny + y) * nx + x); }, z, nz,
                                (wall_mask & 4) != 0)
                    : 0.0f;
}

// Collision of one species at one node, given the mixture, its friction
// vector V and its own moments.  On return P0 holds the new stored rest
// population and F[a] (a >= 1) the stored deviations g_a.  Returns false if a
// result is not finite.
//
// Per direction, with h = f - w rho (the streamed deviation),
//   f~ - w rho = (1 - 1/tau) h + w E(e),
//   E(e) = [ (f^(eq) - w rho)/tau + f^(eq)/c_s^2 (e - u).(du/tau - V)
//            + (1 - 1/(2 tau)) S ] / w,
// with du = u_i^eq - u; the first term is the BGK relaxation toward f^(0)
// (eq. feqi0) written as relaxation toward f^(eq) plus its (e - u).du part,
// the second also carries Omega^ij (eq. Cross_collision_Sirovich).  In the
// projections t = e.u/c_s^2, q = e.(du/tau - V), e.F, e.G of the direction,
// E is a cubic polynomial; its even and odd parts
//   Even = D0 + a2 t^2 + t (ri q + fi e.G)        (+ fi t_i e.R, FRC 2)
//   Odd  = ra t + b2 q + fi e.F + b3 t^2 q
// (ri = rho/c_s^2, fi = (1 - 1/(2 tau))/c_s^2; D0, a2 = ra/2, b2, b3 per
// node) are evaluated once per pair of opposite directions:
// E(+-e) = Even +- Odd.
// FRC 1 adds S_diff: with Theta_i = rho_i V_i,
//   S_diff = w/(2 tau - 1) [(e.u)(e.Theta) - c_s^2 u.Theta]/c_s^4,
// which enters with the same factor (1 - 1/(2 tau)) as S, so the forcing
// bracket e.F - u.F + t e.F becomes (e.F - u.G) + t e.G, G = F + kd Theta.
// FRC 2 also subtracts S_p = w [(e.u)(e.P) - c_s^2 u.P]/c_s^4 with
// P = c_s^2 grad rho_i (so G = F + kd Theta - P) and adds
// S_rho = w w_i [(e.u_i^eq)(e.grad rho) - c_s^2 u_i^eq.grad rho]/c_s^2, i.e.
// the bracket gains t_i e.R - u_i^eq.R with t_i = e.u_i^eq/c_s^2 and
// R = w_i c_s^2 grad rho (w_i = rho_i/rho).
// (1 - 1/tau) h is evaluated as fmaf(-1/tau, h, h): one rounding of an exact
// (1 - 1/tau), so the relaxation keeps f^(eq) as its fixed point; two
// separately rounded coefficients would scale the equilibrium by a constant
// factor every step and drift the composition systematically.
template <int LAT, int FRC>
__device__ __forceinline__ bool collide_species(const SpeciesConst& K, const float (&g)[3],
                                                float rho_i, float dlt_i, const float (&ue_i)[3],
                                                const Mix& M, const float (&V)[3],
                                                const Grads& D, float& P0,
                                                float (&F)[Lat<LAT>::Q]) {
    constexpr int Q = Lat<LAT>::Q;
    constexpr int DIM = Lat<LAT>::DIM;
    using L = Lat<LAT>;
    const float c = K.c, ics = K.ics, itau = K.itau, fp = K.fp;
    // vectors whose projections on a direction give t, q, e.F, e.G (FRC 2:
    // t_i, e.R); components beyond DIM are zero and never projected
    float T[3] = {}, Z[3] = {}, Fc[3] = {}, Gc[3] = {}, Ti[3] = {}, Rc[3] = {};
    float udu = 0.0f, uV = 0.0f, uG = 0.0f, uR = 0.0f;
    const float kr = FRC ? K.kd * rho_i : 0.0f;
    const float wc = FRC == 2 ? rho_i * M.iR * K.cs2 : 0.0f;   // w_i c_s^2
    const float cics = c * ics;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const float du = ue_i[d] - M.U[d];
        const float Fd = rho_i * g[d];
        float Gd = Fd;
        if (FRC) Gd = fmaf(kr, V[d], Gd);
        if (FRC == 2) Gd = fmaf(-K.cs2, D.gi[d], Gd);
        udu = fmaf(M.U[d], du, udu);
        uV = fmaf(M.U[d], V[d], uV);
        uG = fmaf(M.U[d], Gd, uG);
        T[d] = cics * M.U[d];
        Z[d] = c * fmaf(itau, du, -V[d]);
        Fc[d] = c * Fd;
        Gc[d] = c * Gd;
        if (FRC == 2) {
            const float Rd = wc * D.gm[d];
            uR = fmaf(ue_i[d], Rd, uR);
            Ti[d] = cics * ue_i[d];
            Rc[d] = c * Rd;
        }
    }
    const float b0 = -0.5f * M.uu * ics;            // f^(eq)/(w rho) - 1 - t - t^2/2
    const float z0 = fmaf(itau, udu, -uV);          // u.(du/tau - V)
    const float ri = rho_i * ics;
    const float fi = fp * ics;
    const float B = 1.0f + b0;
    const float ra = rho_i * fmaf(-ics, z0, itau);  // rho (1/tau - z0/c_s^2)
    const float D0 = fmaf(itau * rho_i, b0, -fmaf(ri * B, z0, fi * (uG + uR)));
    const float a2 = 0.5f * ra;
    const float b2 = ri * B;
    const float b3 = 0.5f * ri;
    float sgt = 0.0f;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        if (a > L::opp(a)) continue;               // one pass per opposite pair
        const int ab = L::opp(a);
        const float t = cdot<LAT>(a, T[0], T[1], T[2]);
        const float q = cdot<LAT>(a, Z[0], Z[1], Z[2]);
        const float eF = cdot<LAT>(a, Fc[0], Fc[1], Fc[2]);
        const float eG = FRC ? cdot<LAT>(a, Gc[0], Gc[1], Gc[2]) : eF;
        const float t2 = t * t;
        float ev = fmaf(t2, a2, fmaf(t, fmaf(ri, q, fi * eG), D0));
        if (FRC == 2)
            ev = fmaf(fi * cdot<LAT>(a, Ti[0], Ti[1], Ti[2]), cdot<LAT>(a, Rc[0], Rc[1], Rc[2]),
                      ev);
        const float od = fmaf(t, ra, fmaf(q, fmaf(t2, b3, b2), fi * eF));
        const float w = L::w(a);
        const float we = w * ev, wo = w * od;
        const float ha = fmaf(-w, dlt_i, F[a]);
        const float hb = fmaf(-w, dlt_i, F[ab]);
        const float ga = fmaf(-itau, ha, ha) + (we + wo);
        const float gb = fmaf(-itau, hb, hb) + (we - wo);
        F[a] = ga;
        F[ab] = gb;
        sgt += ga + gb;
    }
    float e;
    P0 = store_transform<LAT>(P0, dlt_i, sgt, e);
#pragma unroll
    for (int a = 1; a < Q; ++a) F[a] = fmaf(L::w(a), e, F[a]);
    return isfinite(sgt) && isfinite(P0);
}

// Moving walls (the closing remark of Appendix A).  At a node next to a wall
// moving along itself with velocity u_w, every direction a pointing away from
// the wall gains the paper's term written for the reflected direction,
//   2 w_a rho_i w_i (e_a.u_w)/c_s^2 = 6 w_a rho_i w_i (c_a.u_w)/c,
// with rho_i and the mass fraction w_i of the streamed populations at the
// node (the term adds no mass, so they do not depend on it).  Over the
// reflected directions sum_a w_a c_a c_a = I/18 in the tangential components
// (D2Q9 and D3Q19 alike), so the term raises u_i^eq = c sum_a c_a f_a/rho_i +
// g/2 by w_i u_w/3.
struct WallMove {
    int axis, sigma;   // wall axis; -1 for the low wall, +1 for the high one
    float u[3];
};

// Whether node (x, y, z) lies next to a moving wall; fills W if so.
__device__ __forceinline__ bool moving_wall_at(const LatParams& P, int x, int y, int z,
                                               WallMove& W) {
    const int axis = P.wall_axis;
    if (!P.moving || axis < 0 || axis > 2) return false;
    const int c = axis == 0 ? x : (axis == 1 ? y : z);
    const int n = axis == 0 ? P.nx : (axis == 1 ? P.ny : P.nz);
    int k;
    if (c == 0) k = 0;
    else if (c == n - 1) k = 1;
    else return false;
    W.axis = axis;
    W.sigma = k == 0 ? -1 : 1;
    W.u[0] = P.uw[k][0];
    W.u[1] = P.uw[k][1];
    W.u[2] = P.uw[k][2];
    return W.u[0] != 0.0f || W.u[1] != 0.0f || W.u[2] != 0.0f;
}

// u_i^eq of every species after the moving-wall terms (rho: streamed densities)
template <int NS>
__device__ __forceinline__ void wall_shift_ue(const WallMove& W, const float (&rho)[NS],
                                              float (&ue)[NS][3]) {
    float R = 0.0f;
#pragma unroll
    for (int j = 0; j < NS; ++j) R += rho[j];
    const float iR3 = rcp_nr(R) * (1.0f / 3.0f);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const float wj = rho[j] * iR3;
#pragma unroll
        for (int d = 0; d < 3; ++d) ue[j][d] = fmaf(wj, W.u[d], ue[j][d]);
    }
}

// the moving-wall terms on the streamed deviations of one species (speed c,
// streamed density rho_i, mass fraction w_i); mirror directions get exactly
// opposite terms
template <int LAT>
__device__ __forceinline__ void wall_add_terms(const WallMove& W, float rho_i, float w_i, float c,
                                               float (&F)[Lat<LAT>::Q]) {
    using L = Lat<LAT>;
    const float k = 6.0f * rho_i * w_i * rcp_nr(c);
#pragma unroll
    for (int a = 1; a < L::Q; ++a) {
        const int ca = W.axis == 0 ? L::cx(a) : (W.axis == 1 ? L::cy(a) : L::cz(a));
        if (W.sigma * ca < 0) F[a] = fmaf(L::w(a) * k, cdot<LAT>(a, W.u[0], W.u[1], W.u[2]), F[a]);
    }
}

// Collision of one node, all species, under the specific force g (the
// constant one or the node's value of a force field).  On return P0[s] holds
// the new stored rest population and F[s][a] (a >= 1) the stored deviations
// g_a.  Returns false if a result is not finite.
template <int LAT, int NS, int FRC>
__device__ __forceinline__ bool collide(float (&P0)[NS], float (&F)[NS][Lat<LAT>::Q],
                                        const CollConst& C, const float (&g)[3],
                                        const float (&gi)[NS][3], bool mw, const WallMove& W) {
    float rho[NS], dlt[NS], ue[NS][3];
#pragma unroll
    for (int s = 0; s < NS; ++s) species_moments<LAT>(P0[s], F[s], C.c[s], g, rho[s], dlt[s], ue[s]);
    if (mw) {
        wall_shift_ue<NS>(W, rho, ue);
        float R = 0.0f;
#pragma unroll
        for (int s = 0; s < NS; ++s) R += rho[s];
        const float iR = rcp_nr(R);
#pragma unroll
        for (int s = 0; s < NS; ++s) wall_add_terms<LAT>(W, rho[s], rho[s] * iR, C.c[s], F[s]);
    }
    const Mix M = mixture<NS>(rho, ue, C);
    float y[NS][NS];
    tau_solve<NS>(rho, M.R, M.n, C, y);
    bool ok = isfinite(M.R);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        float V[3];
        friction<NS>(i, rho, ue, y, M.iR, V);
        const SpeciesConst K{C.c[i], C.inv_cs2[i], C.inv_tau[i], C.fpref[i], C.kdiff[i],
                             C.cs2[i]};
        Grads D;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            D.gi[d] = gi[i][d];
            D.gm[d] = 0.0f;
#pragma unroll
            for (int s = 0; s < NS; ++s) D.gm[d] += gi[s][d];
        }
        ok = collide_species<LAT, FRC>(K, g, rho[i], dlt[i], ue[i], M, V, D, P0[i], F[i]) && ok;
    }
    return ok;
}

}  // namespace lbmmc
