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
    // forward recomputation with the intermediates (the reciprocals as in
    // the forward tau_solve: hardware reciprocal plus one Newton step)
    float y[NS][NS], iE[NS][NS], qv[NS], tv[NS], iq[NS];
#pragma unroll
    for (int j = NS - 1; j >= 1; --j) {
        float Rj = 2.0f * R;
#pragma unroll
        for (int s = j + 1; s < NS; ++s) Rj -= rho[s] * y[j][s];
        float q = 0.0f;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            iE[j][i] = rcp_nr(fmaf(n, C.K[i][j], rho[j]));
            q += rho[i] * iE[j][i];
        }
        iq[j] = rcp_nr(1.0f + q);
        const float t = Rj * iq[j];
        qv[j] = q;
        tv[j] = t;
#pragma unroll
        for (int i = 0; i < j; ++i) {
            y[i][j] = t * iE[j][i];
            y[j][i] = y[i][j];
        }
    }
    // reverse, columns in ascending order
#pragma unroll
    for (int j = 1; j < NS; ++j) {
        const float t = tv[j];
        float dt = 0.0f;
        float dE[NS];
#pragma unroll
        for (int i = 0; i < j; ++i) {
            dt += dY[i][j] * iE[j][i];
            dE[i] = -dY[i][j] * t * iE[j][i] * iE[j][i];
        }
        const float dRj = dt * iq[j];
        const float dq = -dt * t * iq[j];
#pragma unroll
        for (int i = 0; i < j; ++i) {
            drho[i] += dq * iE[j][i];
            dE[i] -= dq * rho[i] * iE[j][i] * iE[j][i];
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

// Reverse mode of the collision at one node, in population space, in pieces
// shared by the one-thread-per-node form (collide_vjp) and the
// one-wave-per-species form of the reverse step.  Exact math of the forward
// collision, evaluated directly in FP32 (the adjoint is a linearisation: its
// error enters the gradient, not the state).

// Forward recomputation from the species densities rho and momenta
// jm = sum_a c_a f_a (integer directions) of the streamed populations.
template <int NS>
struct VjpFwd {
    float ue[NS][3];
    bool live[NS];
    float R, n, iR, U[3], UU;
    float y[NS][NS];
};

template <int NS>
__device__ __forceinline__ void vjp_forward(const float (&rho)[NS], const float (&jm)[NS][3],
                                            const CollConst& C, VjpFwd<NS>& f) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        f.live[s] = fabsf(rho[s]) > kRhoTiny;
        const float cr = f.live[s] ? C.c[s] * rcp_nr(rho[s]) : 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) f.ue[s][d] = fmaf(jm[s][d], cr, 0.5f * C.g[d]);
    }
    f.R = 0.0f;
    f.n = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        f.R += rho[s];
        f.n += rho[s] * C.invM[s];
    }
    f.iR = rcp_nr(f.R);
#pragma unroll
    for (int d = 0; d < 3; ++d) f.U[d] = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) f.U[d] += rho[s] * f.ue[s][d] * f.iR;
    tau_solve<NS>(rho, f.R, f.n, C, f.y);
    f.UU = f.U[0] * f.U[0] + f.U[1] * f.U[1] + f.U[2] * f.U[2];
}

// Adjoints of the shared intermediates: u, rho, the species densities and
// equilibrium velocities, and y (dY[i][j] from species i's friction).
template <int NS>
struct VjpAcc {
    float dU[3], dR;
    float drho[NS], due[NS][3];
    float dY[NS][NS];
};

template <int NS>
__device__ __forceinline__ void vjp_zero(VjpAcc<NS>& A) {
    A.dU[0] = A.dU[1] = A.dU[2] = 0.0f;
    A.dR = 0.0f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        A.drho[s] = 0.0f;
        A.due[s][0] = A.due[s][1] = A.due[s][2] = 0.0f;
#pragma unroll
        for (int t = 0; t < NS; ++t) A.dY[s][t] = 0.0f;
    }
}

// Species i's part (i a compile-time index): lt = dL/df~_i on entry, the
// direct term (1 - 1/tau_i) dL/df~_i on return; its terms added to A and
// rho_i dL/dF_i . (dF/dg) to dg.
template <int LAT, int NS>
__device__ __forceinline__ void vjp_species(int i, const float (&rho)[NS], const VjpFwd<NS>& f,
                                            const CollConst& C, float (&lt)[Lat<LAT>::Q],
                                            VjpAcc<NS>& A, float (&dg)[3]) {
    constexpr int Q = Lat<LAT>::Q;
    using L = Lat<LAT>;
    const float c = C.c[i], ics = C.inv_cs2[i], itau = C.inv_tau[i], fp = C.fpref[i];
    const float iR = f.iR;
    // friction V_i = sum_j W_ij (ue_i - ue_j), W_ij = rho_j y_ij / R
    float V[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if (j == i) continue;
        const float w = rho[j] * f.y[i][j] * iR;
#pragma unroll
        for (int d = 0; d < 3; ++d) V[d] += w * (f.ue[i][d] - f.ue[j][d]);
    }
    float du[3], Fv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        du[d] = f.ue[i][d] - f.U[d];
        Fv[d] = rho[i] * C.g[d];
    }
    const float* U = f.U;
    const float uD = U[0] * du[0] + U[1] * du[1] + U[2] * du[2];
    const float uV = U[0] * V[0] + U[1] * V[1] + U[2] * V[2];
    // Every per-direction term of the reverse sweep is lam_a w_a times a
    // polynomial of degree <= 3 in e_a = c (cx, cy, cz): the sweep reduces
    // to the moments of w_a lam_a over the directions.  With integer
    // components in {-1, 0, 1}: n0 = sum w lam, n1_j = sum w lam e_j,
    // n2_jk = sum w lam e_j e_k, n3_jk = sum w lam e_j^2 e_k (j != k); the
    // third moments with three distinct axes vanish on both lattices and
    // e_j^3 = e_j, so the e-moments are c n1, c^2 n2 and c^3 n3 (n1 on the
    // diagonal).  Then, with P_a = beta + ics e.U + ics^2 (e.U)^2 / 2,
    // beta = 1 - ics U.U / 2 and dfeq_a = lam_a (alpha + ics e.Z),
    // alpha = itau (1 - ics u.D) + ics u.V, Z = itau D - V:
    //   PM0 = sum w lam P,  PM1 = sum w lam P e,
    //   drho_i += alpha PM0 + ics Z.PM1, and the vector sums below.
    constexpr int D = L::DIM;
    auto ec = [](int a, int j) { return j == 0 ? L::cx(a) : (j == 1 ? L::cy(a) : L::cz(a)); };
    float n0 = 0.0f, n1[3] = {0.0f, 0.0f, 0.0f}, n2[3][3] = {}, n3[3][3] = {};
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        const float lam = lt[a];
        lt[a] = (1.0f - itau) * lam;
        const float wl = L::w(a) * lam;
        n0 += wl;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (ec(a, j) == 0) continue;
            n1[j] += ec(a, j) > 0 ? wl : -wl;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                if (k == j || ec(a, k) == 0) continue;
                n3[j][k] += ec(a, k) > 0 ? wl : -wl;
                if (k > j) n2[j][k] += ec(a, j) * ec(a, k) > 0 ? wl : -wl;
            }
            n2[j][j] += wl;
        }
    }
    const float c2 = c * c, c3 = c2 * c;
    float M1[3], M2U[3], M2Z[3], M2F[3], M3UU[3], M3ZU[3], Z[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        Z[j] = fmaf(itau, du[j], -V[j]);
        M1[j] = M2U[j] = M2Z[j] = M2F[j] = M3UU[j] = M3ZU[j] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        M1[j] = c * n1[j];
        float u2 = 0.0f, z2 = 0.0f, f2 = 0.0f, uu = n1[j] * U[j] * U[j],
              zu = n1[j] * Z[j] * U[j];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const float m = k == j ? n2[j][j] : (k > j ? n2[j][k] : n2[k][j]);
            u2 = fmaf(m, U[k], u2);
            z2 = fmaf(m, Z[k], z2);
            f2 = fmaf(m, Fv[k], f2);
            if (k == j) continue;
            // M3_jjk and M3_kkj terms
            uu = fmaf(2.0f * n3[j][k], U[j] * U[k], uu);
            uu = fmaf(n3[k][j], U[k] * U[k], uu);
            zu = fmaf(n3[j][k], fmaf(Z[j], U[k], Z[k] * U[j]), zu);
            zu = fmaf(n3[k][j], Z[k] * U[k], zu);
        }
        M2U[j] = c2 * u2;
        M2Z[j] = c2 * z2;
        M2F[j] = c2 * f2;
        M3UU[j] = c3 * uu;
        M3ZU[j] = c3 * zu;
    }
    const float beta = fmaf(-0.5f * ics, f.UU, 1.0f);
    const float alpha = fmaf(itau, fmaf(-ics, uD, 1.0f), ics * uV);
    float UM1 = 0.0f, ZM1 = 0.0f, UM2U = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        UM1 = fmaf(U[j], M1[j], UM1);
        ZM1 = fmaf(Z[j], M1[j], ZM1);
        UM2U = fmaf(U[j], M2U[j], UM2U);
    }
    const float hics2 = 0.5f * ics * ics;
    const float PM0 = fmaf(hics2, UM2U, fmaf(ics, UM1, beta * n0));
    float PM1[3] = {0.0f, 0.0f, 0.0f}, ZPM1 = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        PM1[j] = fmaf(hics2, M3UU[j], fmaf(ics, M2U[j], beta * M1[j]));
        ZPM1 = fmaf(Z[j], PM1[j], ZPM1);
    }
    const float ri = rho[i];
    const float drf = fmaf(ics, ZPM1, alpha * PM0);
    const float s_UU = -0.5f * ics * ri * fmaf(ics, ZM1, alpha * n0);
    const float s_uD = -itau * ics * ri * PM0;
    const float s_uV = ics * ri * PM0;
    const float s_uF = -fp * ics * n0;
    float gU[3], gdu[3], gV[3], gF[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float a1 = fmaf(ics, M2U[j], M1[j]);
        const float a2 = fmaf(ics, M3ZU[j], M2Z[j]);
        gU[j] = fmaf(fp * ics * ics, M2F[j], ri * ics * fmaf(alpha, a1, ics * a2));
        gdu[j] = itau * ics * ri * PM1[j];
        gV[j] = -ics * ri * PM1[j];
        gF[j] = fp * ics * a1;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        gU[d] += s_uD * du[d] + s_uV * V[d] + s_uF * Fv[d] + 2.0f * s_UU * U[d];
        gdu[d] += s_uD * U[d];
        gV[d] += s_uV * U[d];
        gF[d] += s_uF * U[d];
    }
    A.drho[i] += drf;
    // F_i = rho_i g
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.drho[i] += gF[d] * C.g[d];
        dg[d] += rho[i] * gF[d];
    }
    // du_i = ue_i - U
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A.due[i][d] += gdu[d];
        A.dU[d] += gU[d] - gdu[d];
    }
    // V_i = sum_j W_ij (ue_i - ue_j)
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if (j == i) continue;
        const float W = rho[j] * f.y[i][j] * iR;
        float dW = 0.0f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            dW += gV[d] * (f.ue[i][d] - f.ue[j][d]);
            A.due[i][d] += W * gV[d];
            A.due[j][d] -= W * gV[d];
        }
        A.drho[j] += dW * f.y[i][j] * iR;
        A.dY[i][j] += dW * rho[j] * iR;
        A.dR -= dW * W * iR;
    }
}

// Reverse of the mixture velocity, of the cross-relaxation solve and of
// rho = sum rho_s, n = sum rho_s/M_s: completes A.drho and A.due, adds dL/dK.
template <int NS>
__device__ __forceinline__ void vjp_mixture(const float (&rho)[NS], const VjpFwd<NS>& f,
                                            const CollConst& C, VjpAcc<NS>& A,
                                            float (&dK)[NS][NS]) {
    const float iR = f.iR;
    // U = sum_s rho_s ue_s / R
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A.due[s][d] += A.dU[d] * rho[s] * iR;
            A.drho[s] += A.dU[d] * f.ue[s][d] * iR;
        }
    float dR = A.dR - (A.dU[0] * f.U[0] + A.dU[1] * f.U[1] + A.dU[2] * f.U[2]) * iR;
    // y: both orders of a pair are the same unknown
    float dYs[NS][NS];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = 0; j < NS; ++j) dYs[i][j] = i < j ? A.dY[i][j] + A.dY[j][i] : 0.0f;
    float dn = 0.0f;
    tau_vjp<NS>(rho, f.R, f.n, C, dYs, A.drho, dR, dn, dK);
    // R = sum rho, n = sum rho/M
#pragma unroll
    for (int s = 0; s < NS; ++s) A.drho[s] += dR + dn * C.invM[s];
}

// Species s's last part (s compile-time): reverse of ue_s = c_s j_s/rho_s +
// g/2 and of rho_s = sum_a f_a, j_s = sum_a c_a f_a: lt += drho_s + c_s
// c_a . dj_s; dg += due_s/2.
template <int LAT, int NS>
__device__ __forceinline__ void vjp_finish(int s, const float (&rho)[NS], const VjpFwd<NS>& f,
                                           const CollConst& C, const VjpAcc<NS>& A,
                                           float (&lt)[Lat<LAT>::Q], float (&dg)[3]) {
    constexpr int Q = Lat<LAT>::Q;
    using L = Lat<LAT>;
    float dj[3];
    float drho = A.drho[s];
    const float irho = f.live[s] ? rcp_nr(rho[s]) : 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        dg[d] += 0.5f * A.due[s][d];
        dj[d] = A.due[s][d] * irho;
        drho -= A.due[s][d] * (f.ue[s][d] - 0.5f * C.g[d]) * irho;
    }
#pragma unroll
    for (int a = 0; a < Q; ++a)
        lt[a] += drho + C.c[s] * (L::cx(a) * dj[0] + L::cy(a) * dj[1] + L::cz(a) * dj[2]);
}

// Vector-Jacobian product of the collision at one node, all species:
// lt = dL/df~ on entry, dL/df on return; dL/dK_ij and dL/dg accumulated.
template <int LAT, int NS>
__device__ __forceinline__ void collide_vjp(const float (&rho)[NS], const float (&jm)[NS][3],
                                            float (&lt)[NS][Lat<LAT>::Q], const CollConst& C,
                                            float (&dK)[NS][NS], float (&dg)[3]) {
    VjpFwd<NS> f;
    vjp_forward<NS>(rho, jm, C, f);
    VjpAcc<NS> A;
    vjp_zero<NS>(A);
#pragma unroll
    for (int i = 0; i < NS; ++i) vjp_species<LAT, NS>(i, rho, f, C, lt[i], A, dg);
    vjp_mixture<NS>(rho, f, C, A, dK);
#pragma unroll
    for (int s = 0; s < NS; ++s) vjp_finish<LAT, NS>(s, rho, f, C, A, lt[s], dg);
}

}  // namespace lbmmc
