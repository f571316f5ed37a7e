// Data shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmmc {

constexpr int MAXS = 4;

// Per-lattice constants, prepared on the host in double precision and rounded
// once to float.  One entry per lattice of a (possibly batched) context.
struct LatParams {
    int32_t nx, ny, nz, pitch;     // fluid nodes per axis; x-row pitch in floats
    int64_t base;                  // float offset of this lattice in a population buffer
    int64_t plane;                 // floats per (species, direction) plane = nz*ny*pitch
    int64_t field_base;            // node offset of this lattice in dense node fields
    int32_t wall_axis;             // -1: periodic everywhere; 0/1/2: the one wall axis (walls
                                   // at both ends); 3: walls on several axes
    int32_t wall_mask;             // bit a set: walls at both ends of axis a
    int32_t n_species;
    int32_t tile_begin, tile_end;  // this lattice's range in the tile list
    int32_t forcing;               // 0: standard forcing term; 1: plus S_diff; 2: full
    int32_t moving;                // a wall of the wall axis moves (uw nonzero)
    int32_t eqb;                   // 1: the walls are the equilibrium comparison boundary
    float uw[2][3];                // velocities of the low / high wall (tangential)
    float lam[MAXS][3];            // (lambda_-1, lambda_0, lambda_+1) at Courant +c_s;
                                   // the three floats sum to exactly 1
    float c[MAXS];                 // c_s = sqrt(M_1/M_s)
    float inv_cs2[MAXS];           // 1/c_{s,s}^2 = 3/c_s^2
    float inv_tau[MAXS];           // 1/tau_s
    float fpref[MAXS];             // 1 - 1/(2 tau_s)
    float kdiff[MAXS];             // 1/(2 tau_s - 1), the weight of S_diff (forcing >= 1), else 0
    float cs2[MAXS];               // c_{s,s}^2 = c_s^2/3
    float invM[MAXS];              // 1/M_s (normalised masses, M_1 = 1)
    float M[MAXS];                 // normalised masses
    float K[MAXS][MAXS];           // 2 M_i M_j D_ij / (M_1 c_{s,1}^2) = 6 M_i M_j D_ij
    float g[3];                    // specific body force
    float n0;                      // initial total mole number
    double dscale[MAXS][MAXS];     // dK_ij/dD_ij = 6 M_i M_j (adjoint)
};

// One work item of the fused step: a lattice, the origin of a block of
// cross-section columns, and the range [m0, m1) of layers along the slowest
// axis that the block marches through.
struct Tile {
    int32_t lat;
    int32_t x0, y0;
    int32_t m0, m1;
    int32_t pad[3];
};

// Shapes of the species-split kernels: bx * by = 64 (one segment of 64
// columns, any split of them), or W = bx * by / 64 segments of 64 columns
// (bx a multiple of 64) with W <= 4 and ns * W <= 12 (the work-group must
// fit one compute unit at three waves per SIMD).
__host__ __device__ inline bool split_shape_ok(int bx, int by, int ns) {
    if (bx < 1 || by < 1 || (bx * by) % 64) return false;
    const int W = bx * by / 64;
    if (W == 1) return true;
    return bx % 64 == 0 && W <= 4 && ns * W <= 12;
}

// Launch description handed from the host library to the kernel launchers.
struct Launch {
    const float* src;
    float* dst;
    const LatParams* lp;
    const Tile* tiles;
    int32_t ntiles;
    int32_t grid;        // work-groups launched (== ntiles when not persistent)
    int32_t bx, by;      // work-group shape (columns)
    int32_t split;       // 0: one thread per column, all species; 1: one wave per species
    int32_t forcing;     // 0: standard forcing term; 1: plus S_diff; 2: minus S_p plus S_rho
                         // plus S_diff (same for every lattice)
    float* dens;         // forcing 2: species densities of the streamed populations, dense
                         // node fields [lattice][N][nodes] (written by the pre-pass)
    const float* accel;  // force field k(x), dense node fields [lattice][d][nodes], or null
                         // (the constant g of each lattice)
    int32_t moving;      // some lattice has a moving wall
    int32_t eqb;         // the equilibrium comparison boundary (every lattice)
    int32_t wt;          // store populations written through (both buffers fit in the
                         // last-level cache), else non-temporal
    unsigned* flag;      // sticky error flags (bit 0: non-finite)
    hipStream_t stream;
};

// Kernel launchers (defined in the .hip translation units).
hipError_t launch_step(int lattice, int nspecies, const Launch& L);
hipError_t launch_init(int lattice, int nspecies, const LatParams* lp_dev, int lat,
                       const LatParams& lp_host, const double* x0_dev, const float* accel,
                       float* f0_out, float* ft_out, unsigned* flag, hipStream_t s);
hipError_t launch_moments(int lattice, int nspecies, const Launch& L, int direct, float* rho,
                          float* x, float* u, float* ueq, float* us, double* partial, int nq);
hipError_t launch_reduce(const LatParams* lp, int nlat, const double* partial, int nq,
                         double* totals, hipStream_t s);
// adjoint: kernel A (collision VJP into mu, gradient partials per tile),
// kernel B (transposed stream mu -> lam_out), the initialisation VJP, and the
// fixed-order sum of the partials into grad (ng = n_pairs + 3 doubles)
hipError_t launch_adjoint(int lattice, int nspecies, const Launch& L, const float* lam_in,
                          float* mu, double* gpart, int ng);
hipError_t launch_adjoint_stream(int lattice, int nspecies, const Launch& L, const float* mu,
                                 float* lam_out);
// kernel B of a reverse step and kernel A of the step before it in one pass:
// mu_in is the later step's scratch, mu_out this step's
hipError_t launch_adjoint_fused(int lattice, int nspecies, const Launch& L, const float* mu_in,
                                float* mu_out, double* gpart);
hipError_t launch_adjoint_init(int lattice, int nspecies, const LatParams* lp_dev,
                               const LatParams& lp_host, const double* x0, const float* lam0,
                               double* gpart, int nblocks, hipStream_t s);
// mole-fraction profile along x of a stored state (partials per row chunk,
// then a fixed-order sum) and its vector-Jacobian product (single lattice)
hipError_t launch_profile(int lattice, int nspecies, const LatParams* lp_dev,
                          const LatParams& lp_host, const float* state, int rows_per,
                          int nchunks, double* part, double* xbar, hipStream_t s);
// the fixed device array of the allocation-free profile: its size in doubles
// and its address on the current device (looked up once per device)
constexpr int64_t kProfileScratchDoubles = (int64_t)1 << 19;   // 4 MiB
hipError_t profile_scratch(double** out);
hipError_t launch_profile_vjp(int lattice, int nspecies, const LatParams* lp_dev,
                              const LatParams& lp_host, const float* state, const double* dxbar,
                              float* lam, int max_blocks, hipStream_t s);
hipError_t launch_grad_reduce(const LatParams* lp_dev, const double* gpart, int nblocks, int ng,
                              int nspecies, double* grad, hipStream_t s);

}  // namespace lbmmc
