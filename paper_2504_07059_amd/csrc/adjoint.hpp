// Reverse mode of the per-node collision (pure arithmetic, registers only).
#pragma once

#include "collide.hpp"
#include "common.hpp"
#include "lattice.hpp"

namespace lbmmc {

// Reverse mode of tau_solve: given dY (adjoint of the symmetric y, per pair
// summed over both orders), accumulate into drho, dR, dn and dK.
template <int NS>
__device__ __forceinline__ void tau_vjp(const float (&rho)[NS], float R, float n,
                                        const CollConst& C, float (&dY)[NS][NS],
                                        float (&drho)[NS], float& dR, float& dn,
                                        float (&dK)[NS][NS]) {
    // forward recomputation with the intermediates
    float y[NS][NS], E[NS][NS], qv[NS], tv[NS];
#pragma unroll
    for (int j = NS - 1; j >= 1; --j) {
        float Rj = 2.0f * R;
#pragma unroll
        for (int s = j + 1; s < NS; ++s) Rj -= rho[s] * y[j][s];
        float q = 0.0f;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            E[j][i] = fmaf(n, C.K[i][j], rho[j]);
            q += rho[i] / E[j][i];
        }
        const float t = Rj / (1.0f + q);
        qv[j] = q;
        tv[j] = t;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            y[i][j] = t / E[j][i];
            y[j][i] = y[i][j];
        }
    }
    // reverse, columns in ascending order
#pragma unroll
    for (int j = 1; j < NS; ++j) {
        const float t = tv[j], q = qv[j];
        float dt = 0.0f;
        float dE[NS];
#pragma unroll
        for (int i = 0; i < j; ++i) {
            dt += dY[i][j] / E[j][i];
            dE[i] = -dY[i][j] * t / (E[j][i] * E[j][i]);
        }
        const float dRj = dt / (1.0f + q);
        const float dq = -dt * t / (1.0f + q);
#pragma unroll
        for (int i = 0; i < j; ++i) {
            drho[i] += dq / E[j][i];
            dE[i] -= dq * rho[i] / (E[j][i] * E[j][i]);
        }
#pragma unroll
        for (int i = 0; i < j; ++i) {
            drho[j] += dE[i];
            dn += dE[i] * C.K[i][j];
            dK[i][j] += dE[i] * n;
        }
        dR += 2.0f * dRj;
#pragma unroll
        for (int s = j + 1; s < NS; ++s) {
            drho[s] -= dRj * y[j][s];
            dY[j][s] -= dRj * rho[s];
        }
    }
}

// Vector-Jacobian product of the collision at one node, in population space.
// In: the species densities rho and momenta jm = sum_a c_a f_a (integer
// directions) of the streamed populations f; lt = dL/df~.  Out: lt = dL/df;
// dL/dK_ij and dL/dg accumulated.  Exact math of the forward collision,
// evaluated directly in FP32 (the adjoint is a linearisation: its error
// enters the gradient, not the state).
template <int LAT, int NS>
__device__ __forceinline__ void collide_vjp(const float (&rho)[NS], const float (&jm)[NS][3],
                                            float (&lt)[NS][Lat<LAT>::Q], const CollConst& C,
                                            float (&dK)[NS][NS], float (&dg)[3]) {
    constexpr int Q = Lat<LAT>::Q;
    using L = Lat<LAT>;
    // ---------------------------------------------------- forward recomputation
    float ue[NS][3];
    bool live[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        live[s] = fabsf(rho[s]) > kRhoTiny;
        const float cr = live[s] ? C.c[s] / rho[s] : 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) ue[s][d] = fmaf(jm[s][d], cr, 0.5f * C.g[d]);
    }
    float R = 0.0f, n = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        R += rho[s];
        n += rho[s] * C.invM[s];
    }
    const float iR = 1.0f / R;
    float U[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) U[d] += rho[s] * ue[s][d] * iR;
    float y[NS][NS];
    tau_solve<NS>(rho, R, n, C, y);
    float V[NS][3];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
#pragma unroll
        for (int d = 0; d < 3; ++d) V[i][d] = 0.0f;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            if (j == i) continue;
            const float w = rho[j] * y[i][j] * iR;
#pragma unroll
            for (int d = 0; d < 3; ++d) V[i][d] += w * (ue[i][d] - ue[j][d]);
        }
    }
    const float UU = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];

    // ------------------------------------------------------------------ reverse
    float dU[3] = {0.0f, 0.0f, 0.0f}, dR = 0.0f, dn = 0.0f;
    float drho[NS], due[NS][3], dY[NS][NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        drho[s] = 0.0f;
        due[s][0] = due[s][1] = due[s][2] = 0.0f;
#pragma unroll
        for (int t = 0; t < NS; ++t) dY[s][t] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const float c = C.c[i], ics = C.inv_cs2[i], itau = C.inv_tau[i], fp = C.fpref[i];
        float du[3], Fv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            du[d] = ue[i][d] - U[d];
            Fv[d] = rho[i] * C.g[d];
        }
        const float uD = U[0] * du[0] + U[1] * du[1] + U[2] * du[2];
        const float uV = U[0] * V[i][0] + U[1] * V[i][1] + U[2] * V[i][2];
        float gU[3] = {0, 0, 0}, gdu[3] = {0, 0, 0}, gV[3] = {0, 0, 0}, gF[3] = {0, 0, 0};
        float s_uD = 0.0f, s_uV = 0.0f, s_uF = 0.0f, s_UU = 0.0f, drf = 0.0f;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const float ex = c * L::cx(a), ey = c * L::cy(a), ez = c * L::cz(a);
            const float w = L::w(a);
            const float eU = ex * U[0] + ey * U[1] + ez * U[2];
            const float eD = ex * du[0] + ey * du[1] + ez * du[2];
            const float eV = ex * V[i][0] + ey * V[i][1] + ez * V[i][2];
            const float eF = ex * Fv[0] + ey * Fv[1] + ez * Fv[2];
            const float P = 1.0f + ics * eU + 0.5f * ics * ics * eU * eU - 0.5f * ics * UU;
            const float feq = w * rho[i] * P;
            const float lam = lt[i][a];
            lt[i][a] = (1.0f - itau) * lam;
            const float df0 = itau * lam;
            const float dfeq = df0 * (1.0f + ics * (eD - uD)) - lam * ics * (eV - uV);
            const float deD = df0 * feq * ics;
            const float deV = -lam * feq * ics;
            const float dS = fp * lam;
            const float deF = dS * w * ics * (1.0f + ics * eU);
            float deU = dS * w * ics * ics * eF;
            drf += dfeq * w * P;
            const float dP = dfeq * w * rho[i];
            deU += dP * (ics + ics * ics * eU);
            s_UU += -0.5f * ics * dP;
            s_uD -= deD;
            s_uV -= deV;
            s_uF -= dS * w * ics;
            gU[0] += deU * ex; gU[1] += deU * ey; gU[2] += deU * ez;
            gdu[0] += deD * ex; gdu[1] += deD * ey; gdu[2] += deD * ez;
            gV[0] += deV * ex; gV[1] += deV * ey; gV[2] += deV * ez;
            gF[0] += deF * ex; gF[1] += deF * ey; gF[2] += deF * ez;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            gU[d] += s_uD * du[d] + s_uV * V[i][d] + s_uF * Fv[d] + 2.0f * s_UU * U[d];
            gdu[d] += s_uD * U[d];
            gV[d] += s_uV * U[d];
            gF[d] += s_uF * U[d];
        }
        drho[i] += drf;
        // F_i = rho_i g
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            drho[i] += gF[d] * C.g[d];
            dg[d] += rho[i] * gF[d];
        }
        // du_i = ue_i - U
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            due[i][d] += gdu[d];
            dU[d] += gU[d] - gdu[d];
        }
        // V_i = sum_j W_ij (ue_i - ue_j), W_ij = rho_j y_ij / R
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            if (j == i) continue;
            const float W = rho[j] * y[i][j] * iR;
            float dW = 0.0f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                dW += gV[d] * (ue[i][d] - ue[j][d]);
                due[i][d] += W * gV[d];
                due[j][d] -= W * gV[d];
            }
            drho[j] += dW * y[i][j] * iR;
            dY[i][j] += dW * rho[j] * iR;
            dR -= dW * W * iR;
        }
    }
    // U = sum_s rho_s ue_s / R
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            due[s][d] += dU[d] * rho[s] * iR;
            drho[s] += dU[d] * ue[s][d] * iR;
        }
    dR -= (dU[0] * U[0] + dU[1] * U[1] + dU[2] * U[2]) * iR;
    // y: both orders of a pair are the same unknown
    float dYs[NS][NS];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = 0; j < NS; ++j) dYs[i][j] = i < j ? dY[i][j] + dY[j][i] : 0.0f;
    tau_vjp<NS>(rho, R, n, C, dYs, drho, dR, dn, dK);
    // R = sum rho, n = sum rho/M
#pragma unroll
    for (int s = 0; s < NS; ++s) drho[s] += dR + dn * C.invM[s];
    // ue_s = j_s/rho_s + g/2, j_s = c_s sum_a c_a f
    float dj[NS][3];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            dg[d] += 0.5f * due[s][d];
            if (live[s]) {
                dj[s][d] = due[s][d] / rho[s];
                drho[s] -= due[s][d] * (ue[s][d] - 0.5f * C.g[d]) / rho[s];
            } else {
                dj[s][d] = 0.0f;
            }
        }
#pragma unroll
        for (int a = 0; a < Q; ++a)
            lt[s][a] += drho[s] + C.c[s] * (L::cx(a) * dj[s][0] + L::cy(a) * dj[s][1] +
                                             L::cz(a) * dj[s][2]);
    }
}

}  // namespace lbmmc
