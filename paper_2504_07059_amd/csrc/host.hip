// Host side of the C ABI declared in include/lbm_mc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm_mc.h"
#include "common.hpp"

using namespace lbmmc;

namespace {

thread_local std::string g_err;

lbm_mc_status fail(lbm_mc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHECK(expr)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LBM_MC_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                               \
    } while (0)

constexpr int kPitchAlign = 32;   // floats: 128-byte rows
constexpr int kBaseAlign = 64;    // floats: 256-byte lattice bases

int q_of(int lattice) { return lattice == LBM_MC_D2Q9 ? 9 : 19; }
int dim_of(int lattice) { return lattice == LBM_MC_D2Q9 ? 2 : 3; }
int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }
bool is_wall(int32_t bc) { return bc == LBM_MC_WALL || bc == LBM_MC_WALL_EQ; }
bool lattice_has_eq(const lbm_mc_params& q) {
    return q.bc[0] == LBM_MC_WALL_EQ || q.bc[1] == LBM_MC_WALL_EQ || q.bc[2] == LBM_MC_WALL_EQ;
}

// ------------------------------------------------------------ validation
lbm_mc_status validate_params(const lbm_mc_params* p, int32_t L) {
    if (!p) return fail(LBM_MC_ERR_INVALID, "params is NULL");
    if (L < 1) return fail(LBM_MC_ERR_INVALID, "n_lattices must be >= 1 (got %d)", L);
    for (int l = 0; l < L; ++l) {
        const lbm_mc_params& q = p[l];
        if (q.lattice != LBM_MC_D2Q9 && q.lattice != LBM_MC_D3Q19)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: unknown lattice type %d", l, q.lattice);
        if (q.lattice != p[0].lattice || q.n_species != p[0].n_species)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: a batch must share lattice type and species count", l);
        if (q.n_species < 2 || q.n_species > 4)
            return fail(q.n_species > 4 ? LBM_MC_ERR_UNSUPPORTED : LBM_MC_ERR_INVALID,
                        "lattice %d: n_species must be 2..4 (got %d)", l, q.n_species);
        if (q.nx < 1 || q.ny < 1 || q.nz < 1)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: nx, ny, nz must be >= 1", l);
        if (q.lattice == LBM_MC_D2Q9 && q.nz != 1)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: D2Q9 needs nz = 1", l);
        {
            // the kernels address each species' Q planes with 32-bit offsets
            const int64_t pitch = (q.nx + 31) / 32 * 32;
            const int64_t floats = pitch * q.ny * q.nz * (int64_t)(q.lattice == LBM_MC_D2Q9 ? 9 : 19);
            if (floats * 4 >= ((int64_t)1 << 31))
                return fail(LBM_MC_ERR_UNSUPPORTED,
                            "lattice %d: one species' populations exceed 2 GiB per buffer "
                            "(%lld floats); split the lattice", l, (long long)floats);
        }
        int walls = 0, eq_walls = 0;
        for (int a = 0; a < 3; ++a) {
            if (q.bc[a] != LBM_MC_PERIODIC && q.bc[a] != LBM_MC_WALL && q.bc[a] != LBM_MC_WALL_EQ)
                return fail(LBM_MC_ERR_INVALID,
                            "lattice %d: bc[%d] must be PERIODIC, WALL or WALL_EQ", l, a);
            eq_walls += q.bc[a] == LBM_MC_WALL_EQ;
            if (is_wall(q.bc[a])) {
                ++walls;
                const int n = a == 0 ? q.nx : (a == 1 ? q.ny : q.nz);
                if (n < 2)
                    return fail(LBM_MC_ERR_INVALID, "lattice %d: a wall axis needs >= 2 nodes", l);
            }
        }
        if (q.lattice == LBM_MC_D2Q9 && is_wall(q.bc[2]))
            return fail(LBM_MC_ERR_INVALID, "lattice %d: no z walls in 2-D", l);
        if (eq_walls && eq_walls != walls)
            return fail(LBM_MC_ERR_UNSUPPORTED,
                        "lattice %d: WALL and WALL_EQ axes in one lattice are not provided", l);
        if ((eq_walls > 0) != (lattice_has_eq(p[0])))
            return fail(LBM_MC_ERR_UNSUPPORTED,
                        "lattice %d: every lattice of a batch needs the same wall kind", l);
        if (eq_walls && q.forcing != 0)
            return fail(LBM_MC_ERR_UNSUPPORTED,
                        "lattice %d: the equilibrium boundary is provided with forcing 0 only", l);

        const int N = q.n_species;
        for (int i = 0; i < N; ++i) {
            if (!(q.molar_mass[i] > 0.0) || !std::isfinite(q.molar_mass[i]))
                return fail(LBM_MC_ERR_INVALID, "lattice %d: molar_mass[%d] must be > 0", l, i);
            if (i > 0 && q.molar_mass[i] < q.molar_mass[i - 1])
                return fail(LBM_MC_ERR_INVALID,
                            "lattice %d: species must be ordered by ascending molar mass", l);
            for (int j = 0; j < N; ++j) {
                if (i == j) continue;
                const double d = q.diff[i][j], e = q.diff[j][i];
                if (!(d > 0.0) || !std::isfinite(d))
                    return fail(LBM_MC_ERR_INVALID, "lattice %d: diff[%d][%d] must be > 0", l, i, j);
                if (std::fabs(d - e) > 1e-12 * std::fabs(d))
                    return fail(LBM_MC_ERR_INVALID, "lattice %d: diff must be symmetric", l);
            }
        }
        if (!(q.tau1 > 0.5) || !std::isfinite(q.tau1))
            return fail(LBM_MC_ERR_INVALID, "lattice %d: tau1 must be > 1/2 (got %g)", l, q.tau1);
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(q.g[a])) return fail(LBM_MC_ERR_INVALID, "lattice %d: g not finite", l);
        if (q.lattice == LBM_MC_D2Q9 && q.g[2] != 0.0)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: g[2] must be 0 in 2-D", l);
        if (!std::isfinite(q.n0)) return fail(LBM_MC_ERR_INVALID, "lattice %d: n0 not finite", l);
        if (q.forcing < 0 || q.forcing > 2)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: forcing must be 0, 1 or 2", l);
        if (q.forcing == 2)
            for (int a = 0; a < 3; ++a)
                if (is_wall(q.bc[a]) && (a == 0 ? q.nx : (a == 1 ? q.ny : q.nz)) < 3)
                    return fail(LBM_MC_ERR_INVALID,
                                "lattice %d: forcing 2 needs >= 3 nodes on the wall axis", l);
        if (q.forcing != p[0].forcing)
            return fail(LBM_MC_ERR_INVALID, "lattice %d: every lattice needs the same forcing", l);
        if (q.reserved != 0) return fail(LBM_MC_ERR_INVALID, "lattice %d: reserved must be 0", l);
        {
            int wax = -1;
            for (int a = 0; a < 3; ++a)
                if (is_wall(q.bc[a])) wax = a;
            for (int k = 0; k < 2; ++k)
                for (int a = 0; a < 3; ++a) {
                    const double v = q.wall_velocity[k][a];
                    if (!std::isfinite(v))
                        return fail(LBM_MC_ERR_INVALID, "lattice %d: wall velocity not finite", l);
                    if (v == 0.0) continue;
                    if (wax < 0)
                        return fail(LBM_MC_ERR_INVALID,
                                    "lattice %d: a wall velocity needs a wall axis", l);
                    if (walls > 1)
                        return fail(LBM_MC_ERR_UNSUPPORTED,
                                    "lattice %d: moving walls need a single wall axis", l);
                    if (eq_walls)
                        return fail(LBM_MC_ERR_UNSUPPORTED,
                                    "lattice %d: the equilibrium boundary has no moving walls",
                                    l);
                    if (a == wax)
                        return fail(LBM_MC_ERR_INVALID,
                                    "lattice %d: wall velocities must be tangential", l);
                    if (q.lattice == LBM_MC_D2Q9 && a == 2)
                        return fail(LBM_MC_ERR_INVALID, "lattice %d: no z velocity in 2-D", l);
                }
        }
    }
    return LBM_MC_OK;
}

// Normalised problem of one lattice in double precision.
struct Norm {
    int N;
    double M[MAXS], c[MAXS], cs2[MAXS], tau[MAXS], D[MAXS][MAXS], n0;
};

Norm normalise(const lbm_mc_params& q) {
    Norm r{};
    r.N = q.n_species;
    double mmax = 0.0;
    for (int i = 0; i < r.N; ++i) {
        r.M[i] = q.molar_mass[i] / q.molar_mass[0];   // M_1 = 1 (Sec. 4 opening)
        r.c[i] = std::sqrt(1.0 / r.M[i]);             // eq. (speed_DLS)
        r.cs2[i] = r.c[i] * r.c[i] / 3.0;
        r.tau[i] = 0.5 + (q.tau1 - 0.5) * r.M[i];     // common nu (Sec. 3)
        mmax = std::max(mmax, r.M[i]);
        for (int j = 0; j < r.N; ++j) r.D[i][j] = q.diff[i][j];
    }
    r.n0 = q.n0 > 0.0 ? q.n0 : 1.0 / mmax;
    return r;
}

// 1/tau_ij at one node (double), the closed form of the kernel's tau_solve.
void inv_taus(const Norm& nm, const double* rho, double y[MAXS][MAXS]) {
    const int N = nm.N;
    double R = 0.0, n = 0.0;
    for (int i = 0; i < N; ++i) {
        R += rho[i];
        n += rho[i] / nm.M[i];
    }
    for (int i = 0; i < MAXS; ++i)
        for (int j = 0; j < MAXS; ++j) y[i][j] = 0.0;
    for (int j = N - 1; j >= 1; --j) {
        double Rj = 2.0 * R;
        for (int s = j + 1; s < N; ++s) Rj -= rho[s] * y[j][s];
        double E[MAXS], q = 0.0;
        for (int i = 0; i < j; ++i) {
            E[i] = rho[j] + n * 6.0 * nm.M[i] * nm.M[j] * nm.D[i][j];
            q += rho[i] / E[i];
        }
        for (int i = 0; i < j; ++i) y[i][j] = y[j][i] = Rj / (E[i] * (1.0 + q));
    }
}

// Eigenvalues of a small symmetric matrix (cyclic Jacobi).
void sym_eig(int n, double A[MAXS][MAXS], double* ev) {
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i][j] * A[i][j];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (std::fabs(A[p][q]) < 1e-300) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < n; ++i) ev[i] = A[i][i];
}

// Eigenvalue range of the velocity-difference relaxation matrix K at a
// uniform node of composition x (rho_i = x_i M_i n0).  K is similar to the
// symmetric S_ij = -sqrt(rho_i rho_j) y_ij / rho (i != j), S_ii = K_ii.
void k_eig_range(const Norm& nm, const double* x, double& lo, double& hi) {
    const int N = nm.N;
    double rho[MAXS], R = 0.0;
    for (int i = 0; i < N; ++i) {
        rho[i] = x[i] * nm.M[i] * nm.n0;
        R += rho[i];
    }
    double y[MAXS][MAXS];
    inv_taus(nm, rho, y);
    double S[MAXS][MAXS] = {};
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) {
            if (i == j) continue;
            S[i][i] += rho[j] * y[i][j] / R;
            S[i][j] = -std::sqrt(rho[i] * rho[j]) * y[i][j] / R;
        }
    }
    double ev[MAXS];
    sym_eig(N, S, ev);
    lo = ev[0];
    hi = ev[0];
    for (int i = 1; i < N; ++i) {
        lo = std::min(lo, ev[i]);
        hi = std::max(hi, ev[i]);
    }
}

lbm_mc_status validate_x0_and_stability(const lbm_mc_params* p, int32_t L, const double* x0,
                                        double* lam_out) {
    if (!x0) return fail(LBM_MC_ERR_INVALID, "x0 is NULL");
    double worst = 0.0;
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
        const lbm_mc_params& q = p[l];
        const int N = q.n_species;
        const int64_t nodes = (int64_t)q.nx * q.ny * q.nz;
        const double* xl = x0 + off;
        off += nodes * N;
        double mean[MAXS] = {};
        for (int64_t k = 0; k < nodes; ++k) {
            double s = 0.0;
            for (int i = 0; i < N; ++i) {
                const double v = xl[i * nodes + k];
                if (!(v >= 0.0) || !std::isfinite(v))
                    return fail(LBM_MC_ERR_INVALID,
                                "lattice %d: x0 must be finite and >= 0 (node %lld species %d)", l,
                                (long long)k, i);
                s += v;
                mean[i] += v;
            }
            if (std::fabs(s - 1.0) > 1e-9)
                return fail(LBM_MC_ERR_INVALID, "lattice %d: x0 does not sum to 1 at node %lld", l,
                            (long long)k);
        }
        for (int i = 0; i < N; ++i) mean[i] /= (double)nodes;
        const Norm nm = normalise(q);
        // distinct compositions among up to 2048 evenly spaced nodes
        std::set<std::vector<long long>> seen;
        std::vector<std::vector<double>> comps;
        const int64_t stride = std::max<int64_t>(1, nodes / 2048);
        for (int64_t k = 0; k < nodes; k += stride) {
            std::vector<long long> key(N);
            std::vector<double> xs(N);
            for (int i = 0; i < N; ++i) {
                xs[i] = xl[i * nodes + k];
                key[i] = std::llround(xs[i] * 1e9);
            }
            if (seen.insert(key).second) comps.push_back(xs);
        }
        comps.push_back(std::vector<double>(mean, mean + N));
        const double ts[4] = {0.0, 0.25, 0.5, 0.75};
        for (const auto& xs : comps) {
            for (double t : ts) {
                double xt[MAXS];
                for (int i = 0; i < N; ++i) xt[i] = (1.0 - t) * xs[i] + t * mean[i];
                double lo, hi;
                k_eig_range(nm, xt, lo, hi);
                worst = std::max(worst, hi);
                if (hi >= 2.0 || lo < -1e-12) {
                    if (lam_out) *lam_out = hi;
                    return fail(LBM_MC_ERR_UNSTABLE,
                                "lattice %d: cross relaxation is linearly unstable (eigenvalues of K "
                                "in [%g, %g], need [0, 2)); reduce D_ij or the densities",
                                l, lo, hi);
                }
            }
        }
    }
    if (lam_out) *lam_out = worst;
    return LBM_MC_OK;
}

// Interpolation weights of Courant number c rounded to floats whose sum is
// exactly 1: lambda_-1 and lambda_+1 are rounded to the 2^-24 grid, so that
// 1 - lambda_-1 - lambda_+1 is exactly representable.
void exact_triple(double c, float out[3]) {
    const double lm = c * (1.0 + c) / 2.0, lp = -c * (1.0 - c) / 2.0;
    const double grid = std::ldexp(1.0, -24);
    const double a = std::nearbyint(lm / grid) * grid, b = std::nearbyint(lp / grid) * grid;
    out[0] = (float)a;
    out[2] = (float)b;
    out[1] = (float)(1.0 - a - b);
}

struct Layout {
    std::vector<int64_t> base, field;
    std::vector<int32_t> pitch;
    int64_t total = 0;
    int64_t nodes_total = 0;   // fluid nodes of all lattices (dense node fields)
};

Layout make_layout(const lbm_mc_params* p, int32_t L) {
    Layout lo;
    int64_t fb = 0;
    for (int l = 0; l < L; ++l) {
        const auto& q = p[l];
        const int pitch = (int)round_up(q.nx, kPitchAlign);
        lo.pitch.push_back(pitch);
        lo.base.push_back(lo.total);
        lo.field.push_back(fb);
        const int64_t plane = (int64_t)q.nz * q.ny * pitch;
        lo.total = round_up(lo.total + plane * q.n_species * q_of(q.lattice), kBaseAlign);
        fb += (int64_t)q.nx * q.ny * q.nz;
    }
    lo.nodes_total = fb;
    return lo;
}

struct Tuning {
    int bx = 256, by = 1, rows = 32, persistent = 0, split = 0;
};

// Step counts of the captured step sequences that lbm_mc_step replays, longest
// first (both even).  A graph launch costs a few microseconds of its own,
// which is most of a step on a small lattice: on the 1024x64 tube the step
// takes 6.42 us with 32-step graphs and 6.25 us with 512-step ones.
constexpr int kGraphSteps[2] = {512, 32};

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int, int>, Tuning> g_tune_cache;
// (the cache key: lattice, species, nx, ny, nz of the first lattice, lattice count,
// and the kernel specialisation: forcing, force field, moving walls)

}  // namespace

struct lbm_mc_ctx {
    int lattice = 0, N = 0, L = 0, Q = 9, DIM = 2;
    std::vector<lbm_mc_params> params;
    std::vector<LatParams> hlp;
    LatParams* dlp = nullptr;
    Layout layout;
    float* bufA = nullptr;
    float* bufB = nullptr;
    float* cur = nullptr;
    float* prev = nullptr;
    bool prev_valid = false;
    int64_t t = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    unsigned* dflag = nullptr;
    // tiles
    Tuning tune;
    std::vector<Tile> htiles;
    Tile* dtiles = nullptr;
    size_t dtiles_cap = 0;
    double* dpartial = nullptr;
    size_t dpartial_cap = 0;
    double* dtotals = nullptr;
    float* dens = nullptr;              // forcing 2: densities of the streamed populations
    const float* accel = nullptr;       // caller's force field (lbm_mc_init_field), borrowed
    int one_launch = 1;
    int cus = 256;
    // captured step sequences: [length class][which buffer is current]
    hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    // adjoint: scratch population-space buffer, second adjoint buffer for
    // adjoint_run, gradient partials, and the initial mole fractions (kept for
    // the initialisation VJP of single-lattice contexts)
    float* dmu = nullptr;
    float* dlam = nullptr;
    Tile* adj_tiles = nullptr;          // the reverse step's own tile list
    // captured launch sequences of lbm_mc_replay / lbm_mc_adjoint_run, keyed
    // by their arguments
    struct SeqGraph {
        int kind;
        const void *a, *b, *c;
        int64_t n, stride;
        hipGraphExec_t exec;
    };
    std::vector<SeqGraph> seq_graphs;
    int adj_ntiles = 0, adj_bx = 64, adj_by = 1;
    double* dgpart = nullptr;
    size_t dgpart_cap = 0;
    double* dx0 = nullptr;
    // profile partial sums [chunks][N][nx] (allocated on first use)
    double* dprof = nullptr;
    size_t dprof_cap = 0;
    // the fixed scratch array of lbm_mc_profile_static on this context's device
    double* static_scratch = nullptr;
};

namespace {

// The kernel specialisation a context's steps run (the best shape differs:
// the full corrected forcing favours the species-split variant on shapes
// where the plain step does not).
int tune_kind(const lbm_mc_ctx* c) {
    int moving = 0;
    for (const auto& h : c->hlp) moving |= h.moving;
    return c->params[0].forcing + 3 * (c->accel ? 1 : 0) + 6 * moving;
}

void drop_graphs(lbm_mc_ctx* c) {
    for (auto& row : c->gexec)
        for (auto& g : row) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    for (auto& g : c->seq_graphs) (void)hipGraphExecDestroy(g.exec);
    c->seq_graphs.clear();
}

// Sequences longer than this are enqueued directly: a graph of thousands of
// launches (a whole recorded trajectory) is rarely replayed with the same
// buffers, and capturing and instantiating it costs more than the launches.
constexpr int64_t kMaxGraphSequence = 512;

// Run a launch sequence through a captured graph, capturing it on first use
// for this argument set (at most 8 kept).  issue(stream) enqueues the
// kernels; it must not record memsets.
template <class Issue>
lbm_mc_status run_sequence(lbm_mc_ctx* c, int kind, const void* a, const void* b, const void* d,
                           int64_t n, int64_t stride, Issue&& issue) {
    if (n > kMaxGraphSequence) return issue(c->stream);
    for (auto& g : c->seq_graphs)
        if (g.kind == kind && g.a == a && g.b == b && g.c == d && g.n == n && g.stride == stride) {
            HIPCHECK(hipGraphLaunch(g.exec, c->stream));
            return LBM_MC_OK;
        }
    if (c->seq_graphs.size() >= 8) {
        for (auto& g : c->seq_graphs) (void)hipGraphExecDestroy(g.exec);
        c->seq_graphs.clear();
    }
    HIPCHECK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    lbm_mc_status st = issue(c->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (st != LBM_MC_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(LBM_MC_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(LBM_MC_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    c->seq_graphs.push_back({kind, a, b, d, n, stride, exec});
    HIPCHECK(hipGraphLaunch(exec, c->stream));
    return LBM_MC_OK;
}

lbm_mc_status build_tiles(lbm_mc_ctx* c) {
    c->htiles.clear();
    const Tuning& T = c->tune;
    for (int l = 0; l < c->L; ++l) {
        const auto& q = c->params[l];
        const int nm = c->DIM == 2 ? q.ny : q.nz;
        const int nxb = (q.nx + T.bx - 1) / T.bx;
        const int nyb = c->DIM == 3 ? (q.ny + T.by - 1) / T.by : 1;
        const int nmc = (nm + T.rows - 1) / T.rows;
        c->hlp[l].tile_begin = (int)c->htiles.size();
        // layer ranges outermost: the tiles side by side in the cross-section
        // are consecutive in the list, so they run at the same time on one
        // XCD and the x halo one tile reads is the line its neighbour reads in
        // the same layer (2-D: 4 % faster on the 16384x1024 tube, 1 % on the
        // batch; neutral in 3-D)
        for (int mc = 0; mc < nmc; ++mc)
            for (int yb = 0; yb < nyb; ++yb)
                for (int xb = 0; xb < nxb; ++xb) {
                    Tile t{};
                    t.lat = l;
                    t.x0 = xb * T.bx;
                    t.y0 = yb * T.by;
                    // the layers split evenly over the column's nmc tiles
                    // (at most T.rows each): no short last tile
                    t.m0 = (int)((int64_t)mc * nm / nmc);
                    t.m1 = (int)((int64_t)(mc + 1) * nm / nmc);
                    c->htiles.push_back(t);
                }
        c->hlp[l].tile_end = (int)c->htiles.size();
    }
    const size_t nt = c->htiles.size();
    if (nt > c->dtiles_cap) {
        if (c->dtiles) (void)hipFree(c->dtiles);
        c->dtiles = nullptr;
        HIPCHECK(hipMalloc(&c->dtiles, nt * sizeof(Tile)));
        c->dtiles_cap = nt;
    }
    const size_t np = nt * (size_t)(c->N + 3);
    if (np > c->dpartial_cap) {
        if (c->dpartial) (void)hipFree(c->dpartial);
        c->dpartial = nullptr;
        HIPCHECK(hipMalloc(&c->dpartial, np * sizeof(double)));
        c->dpartial_cap = np;
    }
    HIPCHECK(hipMemcpyAsync(c->dtiles, c->htiles.data(), nt * sizeof(Tile), hipMemcpyHostToDevice,
                            c->stream));
    HIPCHECK(hipMemcpyAsync(c->dlp, c->hlp.data(), c->hlp.size() * sizeof(LatParams),
                            hipMemcpyHostToDevice, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    return LBM_MC_OK;
}

// Default execution shape: 64-column tiles, one wave per species, with as
// many layers per tile as keep about eight tiles per compute unit (long
// marches reuse the three-layer register stencil; short ones fill the chip on
// small lattices).
Tuning default_tuning(const lbm_mc_params* p, int n_lattices, int dim, int cus) {
    auto columns = [&](int bx, int by) {
        int64_t n = 0;
        for (int l = 0; l < n_lattices; ++l)
            n += (int64_t)((p[l].nx + bx - 1) / bx) *
                 (dim == 3 ? (p[l].ny + by - 1) / by : 1);
        return n;
    };
    auto layers = [&]() {
        int64_t m = 0;
        for (int l = 0; l < n_lattices; ++l) m = std::max<int64_t>(m, dim == 3 ? p[l].nz : p[l].ny);
        return m;
    };
    // the species-split variant over 64-column rows: as fast as or faster
    // than one thread per column on every workload measured (it keeps several
    // times more waves per SIMD)
    Tuning t;
    t.bx = 64;
    t.by = 1;
    t.split = 1;
    const int64_t cols = columns(t.bx, t.by);
    int64_t rows = cols * layers() / (8 * (int64_t)cus);
    t.rows = (int)std::max<int64_t>(1, std::min<int64_t>(dim == 3 ? 16 : 32, rows));
    t.persistent = 0;
    return t;
}

// work-groups of the grid-stride initialisation VJP
int init_blocks(const lbm_mc_ctx* c) {
    const auto& q = c->params[0];
    const int64_t nodes = (int64_t)q.nx * q.ny * q.nz;
    return (int)std::min<int64_t>((nodes + 255) / 256, (int64_t)c->cus * 8);
}

Launch make_launch(lbm_mc_ctx* c, const float* src, float* dst, hipStream_t s) {
    Launch L{};
    L.src = src;
    L.dst = dst;
    L.lp = c->dlp;
    L.tiles = c->dtiles;
    L.ntiles = (int)c->htiles.size();
    L.grid = c->tune.persistent > 0 ? std::min(L.ntiles, c->tune.persistent) : L.ntiles;
    L.bx = c->tune.bx;
    L.by = c->tune.by;
    L.split = c->tune.split;
    L.forcing = c->params[0].forcing;
    L.dens = c->dens;
    L.accel = c->accel;
    L.moving = 0;
    for (const auto& h : c->hlp) L.moving |= h.moving;
    L.eqb = c->hlp[0].eqb;
    // both population buffers within the 256 MB last-level cache: the stores
    // write through to it (the next step reads them back from there); above
    // it they stream past the caches
    L.wt = 2 * c->layout.total * (int64_t)sizeof(float) <= ((int64_t)256 << 20) ? 1 : 0;
    L.flag = c->dflag;
    L.stream = s;
    return L;
}

// One step from src to dst (all lattices).
lbm_mc_status launch_one(lbm_mc_ctx* c, const float* src, float* dst, hipStream_t s) {
    if (c->L > 1 && !c->one_launch) {
        for (int l = 0; l < c->L; ++l) {
            Launch L = make_launch(c, src, dst, s);
            L.tiles = c->dtiles + c->hlp[l].tile_begin;
            L.ntiles = c->hlp[l].tile_end - c->hlp[l].tile_begin;
            L.grid = L.ntiles;
            HIPCHECK(launch_step(c->lattice, c->N, L));
        }
        return LBM_MC_OK;
    }
    HIPCHECK(launch_step(c->lattice, c->N, make_launch(c, src, dst, s)));
    return LBM_MC_OK;
}

// The long step sequences only where a step is one launch (a batch stepped
// with one launch per lattice would put hundreds of thousands of nodes in one
// graph).
bool long_graphs(const lbm_mc_ctx* c) { return c->L == 1 || c->one_launch; }

lbm_mc_status get_graph(lbm_mc_ctx* c, int cls, hipGraphExec_t* out) {
    const int key = c->cur == c->bufA ? 0 : 1;
    if (!c->gexec[cls][key]) {
        HIPCHECK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        float* src = c->cur;
        float* dst = c->prev;
        lbm_mc_status st = LBM_MC_OK;
        for (int i = 0; i < kGraphSteps[cls] && st == LBM_MC_OK; ++i) {
            st = launch_one(c, src, dst, c->cap);
            std::swap(src, dst);
        }
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap, &g);
        if (st != LBM_MC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(LBM_MC_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&c->gexec[cls][key], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return fail(LBM_MC_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    *out = c->gexec[cls][key];
    return LBM_MC_OK;
}

lbm_mc_status check_flag(lbm_mc_ctx* c) {
    unsigned f = 0;
    HIPCHECK(hipMemcpyAsync(&f, c->dflag, sizeof f, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    if (f & 1u)
        return fail(LBM_MC_ERR_NONFINITE,
                    "a step produced a non-finite population (unstable parameters or input)");
    return LBM_MC_OK;
}

// Tiles of the reverse step: 64 columns (64 x 1 in 2-D, 32 x 2 in 3-D, one
// wave per species), layers per tile chosen for about eight tiles per
// compute unit.
lbm_mc_status build_adj_tiles(lbm_mc_ctx* c) {
    const auto& q = c->params[0];
    const int bx = c->DIM == 3 ? 32 : 64, by = c->DIM == 3 ? 2 : 1;
    const int nm = c->DIM == 2 ? q.ny : q.nz;
    const int nxb = (q.nx + bx - 1) / bx, nyb = c->DIM == 3 ? (q.ny + by - 1) / by : 1;
    const int64_t cols = (int64_t)nxb * nyb;
    const int rows = (int)std::max<int64_t>(1, std::min<int64_t>(16, cols * nm / (8 * (int64_t)c->cus)));
    std::vector<Tile> h;
    for (int xb = 0; xb < nxb; ++xb)
        for (int yb = 0; yb < nyb; ++yb)
            for (int m0 = 0; m0 < nm; m0 += rows) {
                Tile t{};
                t.lat = 0;
                t.x0 = xb * bx;
                t.y0 = yb * by;
                t.m0 = m0;
                t.m1 = std::min(nm, m0 + rows);
                h.push_back(t);
            }
    HIPCHECK(hipMalloc(&c->adj_tiles, h.size() * sizeof(Tile)));
    HIPCHECK(hipMemcpyAsync(c->adj_tiles, h.data(), h.size() * sizeof(Tile), hipMemcpyHostToDevice,
                            c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
    c->adj_ntiles = (int)h.size();
    c->adj_bx = bx;
    c->adj_by = by;
    return LBM_MC_OK;
}

lbm_mc_status adjoint_prepare(lbm_mc_ctx* c) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (c->L != 1) return fail(LBM_MC_ERR_UNSUPPORTED, "adjoint: batched contexts are not supported");
    if (c->params[0].forcing != 0)
        return fail(LBM_MC_ERR_UNSUPPORTED, "adjoint: only forcing = 0 is differentiated");
    if (c->accel)
        return fail(LBM_MC_ERR_UNSUPPORTED, "adjoint: a force-field context is not differentiated");
    if (c->hlp[0].moving)
        return fail(LBM_MC_ERR_UNSUPPORTED, "adjoint: moving walls are not differentiated");
    if (c->hlp[0].wall_axis > 2)
        return fail(LBM_MC_ERR_UNSUPPORTED, "adjoint: walls on several axes are not differentiated");
    if (c->hlp[0].eqb)
        return fail(LBM_MC_ERR_UNSUPPORTED,
                    "adjoint: the equilibrium boundary is not differentiated");
    const size_t bytes = (size_t)c->layout.total * sizeof(float);
    if (!c->dmu) {
        HIPCHECK(hipMalloc(&c->dmu, bytes));
        HIPCHECK(hipMemsetAsync(c->dmu, 0, bytes, c->stream));
    }
    if (!c->adj_tiles) {
        lbm_mc_status st = build_adj_tiles(c);
        if (st != LBM_MC_OK) return st;
    }
    const size_t ng = (size_t)(c->N * (c->N - 1) / 2 + 3);
    const size_t need = ng * std::max((size_t)c->adj_ntiles, (size_t)init_blocks(c));
    if (need > c->dgpart_cap) {
        if (c->dgpart) (void)hipFree(c->dgpart);
        c->dgpart = nullptr;
        HIPCHECK(hipMalloc(&c->dgpart, need * sizeof(double)));
        c->dgpart_cap = need;
    }
    return LBM_MC_OK;
}

// Row chunks of the profile reduction: enough work-groups to fill the chip
// (about 2048 of 64 columns), each chunk at least one row.
void profile_chunks(const lbm_mc_ctx* c, int& rows_per, int& nchunks) {
    const auto& q = c->params[0];
    const int64_t rows = (int64_t)q.ny * q.nz;
    const int64_t xb = (q.nx + 63) / 64;
    int64_t want = std::max<int64_t>(1, std::min<int64_t>(rows, (2048 + xb - 1) / xb));
    rows_per = (int)((rows + want - 1) / want);
    nchunks = (int)((rows + rows_per - 1) / rows_per);
}

lbm_mc_status profile_check(lbm_mc_ctx* c, const float* state, const void* out) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (c->L != 1)
        return fail(LBM_MC_ERR_UNSUPPORTED, "profile: batched contexts are not supported");
    if (!state || !out) return fail(LBM_MC_ERR_INVALID, "profile: NULL buffer");
    return LBM_MC_OK;
}

// states: n buffers of the population layout at a stride of `stride` floats
lbm_mc_status check_sequence(lbm_mc_ctx* c, const float* states, int64_t n, int64_t stride) {
    if (n == 0) return LBM_MC_OK;
    if (stride < c->layout.total)
        return fail(LBM_MC_ERR_INVALID, "stride %lld below the buffer size %lld", (long long)stride,
                    (long long)c->layout.total);
    if (stride % 4 || (uintptr_t)states % 16)
        return fail(LBM_MC_ERR_INVALID, "state sequence must be 16-byte aligned (stride % 4 == 0)");
    return LBM_MC_OK;
}

// Per-tile FP64 gradient partials: cleared before a sequence of reverse steps,
// accumulated by every kernel A of the sequence, summed into grad once.
lbm_mc_status grad_clear(lbm_mc_ctx* c, int nblocks) {
    const size_t ng = (size_t)(c->N * (c->N - 1) / 2 + 3);
    HIPCHECK(hipMemsetAsync(c->dgpart, 0, ng * nblocks * sizeof(double), c->stream));
    return LBM_MC_OK;
}

lbm_mc_status grad_sum(lbm_mc_ctx* c, int nblocks, double* grad) {
    const int ng = c->N * (c->N - 1) / 2 + 3;
    HIPCHECK(launch_grad_reduce(c->dlp, c->dgpart, nblocks, ng, c->N, grad, c->stream));
    return LBM_MC_OK;
}

Launch adjoint_launch(lbm_mc_ctx* c, const float* f_prev, hipStream_t stream) {
    Launch L = make_launch(c, f_prev, nullptr, stream);
    L.tiles = c->adj_tiles;
    L.ntiles = L.grid = c->adj_ntiles;
    L.bx = c->adj_bx;
    L.by = c->adj_by;
    // the reverse step keeps four population-sized buffers in play (the
    // state, the two adjoints and the scratch): written-through stores while
    // they fit in the last-level cache
    L.wt = 4 * c->layout.total * (int64_t)sizeof(float) <= ((int64_t)256 << 20) ? 1 : 0;
    return L;
}

// kernel A (partials accumulated per tile), kernel B
lbm_mc_status adjoint_one(lbm_mc_ctx* c, const float* f_prev, const float* lam_in,
                          float* lam_out, hipStream_t stream) {
    const int ng = c->N * (c->N - 1) / 2 + 3;
    const Launch L = adjoint_launch(c, f_prev, stream);
    HIPCHECK(launch_adjoint(c->lattice, c->N, L, lam_in, c->dmu, c->dgpart, ng));
    HIPCHECK(launch_adjoint_stream(c->lattice, c->N, L, c->dmu, lam_out));
    return LBM_MC_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* lbm_mc_last_error(void) { return g_err.c_str(); }

lbm_mc_status lbm_mc_layout(const lbm_mc_params* p, int32_t n_lattices, int64_t* buffer_floats,
                            int64_t* lattice_offsets, int32_t* pitch, int64_t* field_offsets) {
    lbm_mc_status st = validate_params(p, n_lattices);
    if (st != LBM_MC_OK) return st;
    if (!buffer_floats) return fail(LBM_MC_ERR_INVALID, "buffer_floats is NULL");
    Layout lo = make_layout(p, n_lattices);
    *buffer_floats = lo.total;
    for (int l = 0; l < n_lattices; ++l) {
        if (lattice_offsets) lattice_offsets[l] = lo.base[l];
        if (pitch) pitch[l] = lo.pitch[l];
        if (field_offsets) field_offsets[l] = lo.field[l];
    }
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_check(const lbm_mc_params* p, int32_t n_lattices, const double* x0,
                           double* lambda_max) {
    lbm_mc_status st = validate_params(p, n_lattices);
    if (st != LBM_MC_OK) return st;
    return validate_x0_and_stability(p, n_lattices, x0, lambda_max);
}

static lbm_mc_status init_impl(const lbm_mc_params* p, int32_t n_lattices, const double* x0,
                               const float* accel, float* f_a, float* f_b,
                               int64_t buffer_floats, void* hip_stream, lbm_mc_ctx** out) {
    if (!out) return fail(LBM_MC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    lbm_mc_status st = lbm_mc_check(p, n_lattices, x0, nullptr);
    if (st != LBM_MC_OK) return st;
    if (accel) {
        if ((uintptr_t)accel % 4)
            return fail(LBM_MC_ERR_INVALID, "the force field must be 4-byte aligned");
        if (lattice_has_eq(p[0]))
            return fail(LBM_MC_ERR_UNSUPPORTED,
                        "a force field with the equilibrium boundary is not provided");
        for (int l = 0; l < n_lattices; ++l)
            for (int k = 0; k < 2; ++k)
                for (int a = 0; a < 3; ++a)
                    if (p[l].wall_velocity[k][a] != 0.0)
                        return fail(LBM_MC_ERR_UNSUPPORTED,
                                    "lattice %d: a force field with moving walls is not provided",
                                    l);
        for (int l = 0; l < n_lattices; ++l)
            if (p[l].g[0] != 0.0 || p[l].g[1] != 0.0 || p[l].g[2] != 0.0)
                return fail(LBM_MC_ERR_INVALID,
                            "lattice %d: g must be 0 when a force field is given", l);
    }
    if (!f_a || !f_b) return fail(LBM_MC_ERR_INVALID, "population buffers must not be NULL");
    if (f_a == f_b) return fail(LBM_MC_ERR_INVALID, "f_a and f_b must be distinct buffers");
    Layout lo = make_layout(p, n_lattices);
    if (buffer_floats < lo.total)
        return fail(LBM_MC_ERR_INVALID, "buffers hold %lld floats, %lld needed",
                    (long long)buffer_floats, (long long)lo.total);
    const uintptr_t a0 = (uintptr_t)f_a, a1 = (uintptr_t)f_b;
    const uintptr_t bytes = (uintptr_t)lo.total * sizeof(float);
    if (a0 < a1 + bytes && a1 < a0 + bytes)
        return fail(LBM_MC_ERR_INVALID, "f_a and f_b overlap");
    if ((a0 | a1) % 16)
        return fail(LBM_MC_ERR_INVALID, "population buffers must be 16-byte aligned");

    auto* c = new lbm_mc_ctx();
    c->lattice = p[0].lattice;
    c->N = p[0].n_species;
    c->L = n_lattices;
    c->Q = q_of(c->lattice);
    c->DIM = dim_of(c->lattice);
    c->params.assign(p, p + n_lattices);
    c->accel = accel;
    c->layout = lo;
    c->bufA = f_a;
    c->bufB = f_b;
    c->cur = f_a;
    c->prev = f_b;
    c->stream = (hipStream_t)hip_stream;
    auto bail = [&](lbm_mc_status s) {
        std::string keep = g_err;
        lbm_mc_destroy(c);
        g_err = keep;
        return s;
    };
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return bail(fail(LBM_MC_ERR_HIP, "no HIP device"));
    (void)hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (profile_scratch(&c->static_scratch) != hipSuccess)
        return bail(fail(LBM_MC_ERR_HIP, "device address of the profile scratch"));
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(LBM_MC_ERR_HIP, "stream create failed"));

    // per-lattice constants
    c->hlp.resize(n_lattices);
    for (int l = 0; l < n_lattices; ++l) {
        const auto& q = p[l];
        const Norm nm = normalise(q);
        LatParams& P = c->hlp[l];
        memset(&P, 0, sizeof P);
        P.nx = q.nx; P.ny = q.ny; P.nz = q.nz;
        P.pitch = lo.pitch[l];
        P.base = lo.base[l];
        P.plane = (int64_t)q.nz * q.ny * lo.pitch[l];
        P.field_base = lo.field[l];
        P.wall_axis = -1;
        P.wall_mask = 0;
        P.eqb = lattice_has_eq(q) ? 1 : 0;
        for (int a = 0; a < 3; ++a)
            if (is_wall(q.bc[a])) {
                P.wall_axis = P.wall_mask ? 3 : a;
                P.wall_mask |= 1 << a;
            }
        P.n_species = q.n_species;
        P.forcing = q.forcing;
        P.moving = 0;
        for (int k = 0; k < 2; ++k)
            for (int a = 0; a < 3; ++a) {
                P.uw[k][a] = (float)q.wall_velocity[k][a];
                if (q.wall_velocity[k][a] != 0.0) P.moving = 1;
            }
        for (int i = 0; i < MAXS; ++i) {
            if (i < nm.N) {
                exact_triple(nm.c[i], P.lam[i]);
                P.c[i] = (float)nm.c[i];
                P.inv_cs2[i] = (float)(1.0 / nm.cs2[i]);
                P.inv_tau[i] = (float)(1.0 / nm.tau[i]);
                P.fpref[i] = (float)(1.0 - 0.5 / nm.tau[i]);
                P.kdiff[i] = q.forcing >= 1 ? (float)(1.0 / (2.0 * nm.tau[i] - 1.0)) : 0.0f;
                P.cs2[i] = (float)nm.cs2[i];
                P.invM[i] = (float)(1.0 / nm.M[i]);
                P.M[i] = (float)nm.M[i];
                for (int j = 0; j < nm.N; ++j) {
                    const double k = i == j ? 0.0 : 6.0 * nm.M[i] * nm.M[j] * nm.D[i][j];
                    P.K[i][j] = (float)k;
                    P.dscale[i][j] = i == j ? 0.0 : 6.0 * nm.M[i] * nm.M[j];
                }
            }
        }
        for (int a = 0; a < 3; ++a) P.g[a] = (float)q.g[a];
        P.n0 = (float)nm.n0;
    }
    if (hipMalloc(&c->dlp, n_lattices * sizeof(LatParams)) != hipSuccess ||
        hipMalloc(&c->dflag, sizeof(unsigned)) != hipSuccess ||
        hipMalloc(&c->dtotals, (size_t)n_lattices * (c->N + 3) * sizeof(double)) != hipSuccess ||
        (p[0].forcing == 2 &&
         hipMalloc(&c->dens, (size_t)lo.nodes_total * c->N * sizeof(float)) != hipSuccess))
        return bail(fail(LBM_MC_ERR_HIP, "device allocation failed"));
    if (hipMemsetAsync(c->dflag, 0, sizeof(unsigned), c->stream) != hipSuccess)
        return bail(fail(LBM_MC_ERR_HIP, "memset failed"));

    // default execution shape, or a cached autotuned one
    Tuning t = default_tuning(p, n_lattices, c->DIM, c->cus);
    if (lattice_has_eq(p[0])) {
        t.split = 0;   // the equilibrium boundary runs one thread per column
    } else {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(
            {c->lattice, c->N, p[0].nx, p[0].ny, p[0].nz, n_lattices, tune_kind(c)});
        if (it != g_tune_cache.end()) t = it->second;
    }
    c->tune = t;
    st = build_tiles(c);
    if (st != LBM_MC_OK) return bail(st);

    // initial state: f(0) into f_b, f~(0) into f_a
    double* dx0 = nullptr;
    int64_t nx0 = 0;
    for (int l = 0; l < n_lattices; ++l) nx0 += (int64_t)p[l].nx * p[l].ny * p[l].nz * c->N;
    if (hipMalloc(&dx0, nx0 * sizeof(double)) != hipSuccess)
        return bail(fail(LBM_MC_ERR_HIP, "x0 staging allocation failed"));
    hipError_t e = hipMemcpyAsync(dx0, x0, nx0 * sizeof(double), hipMemcpyHostToDevice, c->stream);
    for (int l = 0; l < n_lattices && e == hipSuccess; ++l)
        e = launch_init(c->lattice, c->N, c->dlp, l, c->hlp[l], dx0, accel, c->prev, c->cur,
                        c->dflag, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (n_lattices == 1)
        c->dx0 = dx0;
    else
        (void)hipFree(dx0);
    if (e != hipSuccess) return bail(fail(LBM_MC_ERR_HIP, "init: %s", hipGetErrorString(e)));
    c->prev_valid = true;
    c->t = 0;
    st = check_flag(c);
    if (st != LBM_MC_OK) return bail(st);
    *out = c;
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_init(const lbm_mc_params* p, int32_t n_lattices, const double* x0, float* f_a,
                          float* f_b, int64_t buffer_floats, void* hip_stream, lbm_mc_ctx** out) {
    return init_impl(p, n_lattices, x0, nullptr, f_a, f_b, buffer_floats, hip_stream, out);
}

lbm_mc_status lbm_mc_init_field(const lbm_mc_params* p, int32_t n_lattices, const double* x0,
                                const float* accel, float* f_a, float* f_b,
                                int64_t buffer_floats, void* hip_stream, lbm_mc_ctx** out) {
    if (!accel) {
        if (out) *out = nullptr;
        return fail(LBM_MC_ERR_INVALID, "accel is NULL");
    }
    return init_impl(p, n_lattices, x0, accel, f_a, f_b, buffer_floats, hip_stream, out);
}

lbm_mc_status lbm_mc_step(lbm_mc_ctx* c, int64_t n) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (n < 0) return fail(LBM_MC_ERR_INVALID, "n_steps must be >= 0");
    while (n > 0) {
        const int cls = n >= kGraphSteps[0] && long_graphs(c) ? 0
                        : (n >= kGraphSteps[1] ? 1 : -1);
        if (cls >= 0) {
            hipGraphExec_t g;
            lbm_mc_status st = get_graph(c, cls, &g);
            if (st != LBM_MC_OK) return st;
            HIPCHECK(hipGraphLaunch(g, c->stream));
            n -= kGraphSteps[cls];
            c->t += kGraphSteps[cls];   // an even count: cur/prev are back in place
        } else {
            lbm_mc_status st = launch_one(c, c->cur, c->prev, c->stream);
            if (st != LBM_MC_OK) return st;
            std::swap(c->cur, c->prev);
            c->t += 1;
            n -= 1;
        }
        c->prev_valid = true;
    }
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_prepare(lbm_mc_ctx* c, int64_t n) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (n < 0) return fail(LBM_MC_ERR_INVALID, "n_steps must be >= 0");
    // the graph lengths are even, so lbm_mc_step replays them all with the
    // current buffer assignment
    for (int cls = 0; cls < 2; ++cls) {
        if (n < kGraphSteps[cls] || (cls == 0 && !long_graphs(c))) continue;
        hipGraphExec_t g;
        lbm_mc_status st = get_graph(c, cls, &g);
        if (st != LBM_MC_OK) return st;
        n %= kGraphSteps[cls];
    }
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_sync(lbm_mc_ctx* c) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    return check_flag(c);
}

lbm_mc_status lbm_mc_moments(lbm_mc_ctx* c, float* rho, float* x, float* u, float* ueq,
                             float* us, double* mass, double* momentum) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (!c->prev_valid)
        return fail(LBM_MC_ERR_INVALID, "moments need f~(t-1): restore it or take one step");
    const int nq = c->N + 3;
    Launch L = make_launch(c, c->prev, nullptr, c->stream);
    if (c->tune.bx * c->tune.by % 64) return fail(LBM_MC_ERR_INVALID, "block size must be a multiple of 64");
    HIPCHECK(launch_moments(c->lattice, c->N, L, c->t == 0 ? 1 : 0, rho, x, u, ueq, us,
                            c->dpartial, nq));
    if (mass || momentum) {
        HIPCHECK(launch_reduce(c->dlp, c->L, c->dpartial, nq, c->dtotals, c->stream));
        std::vector<double> h((size_t)c->L * nq);
        HIPCHECK(hipMemcpyAsync(h.data(), c->dtotals, h.size() * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream));
        HIPCHECK(hipStreamSynchronize(c->stream));
        for (int l = 0; l < c->L; ++l) {
            if (mass)
                for (int s = 0; s < c->N; ++s) mass[l * c->N + s] = h[(size_t)l * nq + s];
            if (momentum)
                for (int d = 0; d < c->DIM; ++d) momentum[l * c->DIM + d] = h[(size_t)l * nq + c->N + d];
        }
        return check_flag(c);
    }
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_state(lbm_mc_ctx* c, float** cur, float** prev, int64_t* t) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (cur) *cur = c->cur;
    if (prev) *prev = c->prev;
    if (t) *t = c->t;
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_restore(lbm_mc_ctx* c, const float* cur, const float* prev, int64_t t) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (!cur) return fail(LBM_MC_ERR_INVALID, "cur is NULL");
    if (t < 0) return fail(LBM_MC_ERR_INVALID, "t must be >= 0");
    const size_t bytes = (size_t)c->layout.total * sizeof(float);
    if (cur != c->cur) HIPCHECK(hipMemcpyAsync(c->cur, cur, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (prev && prev != c->prev)
        HIPCHECK(hipMemcpyAsync(c->prev, prev, bytes, hipMemcpyDeviceToDevice, c->stream));
    c->prev_valid = prev != nullptr;
    c->t = t;
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_set_tuning(lbm_mc_ctx* c, int32_t bx, int32_t by, int32_t rows,
                                int32_t persistent, int32_t variant) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    Tuning t = c->tune;
    if (bx) t.bx = bx;
    if (by) t.by = by;
    if (rows) t.rows = rows;
    if (persistent >= 0) t.persistent = persistent;
    if (variant >= 0) t.split = variant;
    else if (!split_shape_ok(t.bx, t.by, c->N)) t.split = 0;   // keep it if the shape allows
    if (t.split != 0 && t.split != 1) return fail(LBM_MC_ERR_INVALID, "variant must be 0 or 1");
    if (t.bx < 8 || t.bx > 256 || t.bx % 8) return fail(LBM_MC_ERR_INVALID, "block_x must be 8..256, multiple of 8");
    if (c->DIM == 2 && t.by != 1) return fail(LBM_MC_ERR_INVALID, "block_y must be 1 in 2-D");
    if (t.by < 1 || t.bx * t.by > 256 || (t.bx * t.by) % 64)
        return fail(LBM_MC_ERR_INVALID, "block_x*block_y must be 64, 128, 192 or 256");
    if (t.split && !split_shape_ok(t.bx, t.by, c->N))
        return fail(LBM_MC_ERR_INVALID,
                    "the species-split variant needs block_x*block_y = 64, or W = "
                    "block_x*block_y/64 segments of 64 columns (block_x a multiple of 64) with "
                    "N*W <= 12");
    if (t.split && c->hlp[0].eqb)
        return fail(LBM_MC_ERR_UNSUPPORTED,
                    "the equilibrium boundary runs execution variant 0 only");
    if (t.rows < 1) return fail(LBM_MC_ERR_INVALID, "rows must be >= 1");
    c->tune = t;
    return build_tiles(c);
}

lbm_mc_status lbm_mc_get_tuning(lbm_mc_ctx* c, int32_t* bx, int32_t* by, int32_t* rows,
                                int32_t* persistent, int32_t* variant) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (bx) *bx = c->tune.bx;
    if (by) *by = c->tune.by;
    if (rows) *rows = c->tune.rows;
    if (persistent) *persistent = c->tune.persistent;
    if (variant) *variant = c->tune.split;
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_autotune(lbm_mc_ctx* c, int32_t reps, double* best_us) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (reps < 1) return fail(LBM_MC_ERR_INVALID, "reps must be >= 1");
    std::vector<Tuning> cands;
    int nm = 0;
    for (const auto& q : c->params) nm = std::max(nm, c->DIM == 2 ? q.ny : q.nz);
    const int rowsv[] = {1, 2, 4, 8, 12, 16, 24, 32, 64, 128};
    if (c->DIM == 2) {
        for (int bx : {64, 128, 256})
            for (int r : rowsv)
                for (int ps : {0, 1}) {
                    if (r > 2 * nm && r != 1) continue;
                    Tuning t;
                    t.bx = bx; t.by = 1; t.rows = r;
                    t.persistent = ps ? c->cus * (1024 / bx) : 0;
                    cands.push_back(t);
                }
        for (int bx : {64, 128, 192, 256})
            for (int r : rowsv)
                for (int ps : {0, 1}) {
                    if (r > 2 * nm && r != 1) continue;
                    if (!split_shape_ok(bx, 1, c->N)) continue;
                    if (bx > 64 && ps) continue;
                    Tuning t;
                    t.bx = bx; t.by = 1; t.rows = r; t.split = 1;
                    t.persistent = ps ? c->cus * 8 : 0;
                    cands.push_back(t);
                }
    } else {
        for (int bx : {32, 64, 128})
            for (int by : {1, 2, 4, 8})
                for (int r : {8, 16, 32, 64}) {
                    if (bx * by < 64 || bx * by > 256) continue;
                    if (r > 2 * nm && r != 8) continue;
                    Tuning t;
                    t.bx = bx; t.by = by; t.rows = r; t.persistent = 0;
                    cands.push_back(t);
                }
        for (int bx : {16, 32, 64})
            for (int r : {4, 8, 16, 32, 64}) {
                if (r > 2 * nm && r != 4) continue;
                Tuning t;
                t.bx = bx; t.by = 64 / bx; t.rows = r; t.persistent = 0; t.split = 1;
                cands.push_back(t);
            }
        // several y rows of 64 columns per work-group
        for (int by : {2, 3, 4})
            for (int r : {8, 16, 32}) {
                if (r > 2 * nm && r != 8) continue;
                if (!split_shape_ok(64, by, c->N)) continue;
                Tuning t;
                t.bx = 64; t.by = by; t.rows = r; t.persistent = 0; t.split = 1;
                cands.push_back(t);
            }
    }
    // the candidates write f~ into prev: from the first launch on it no
    // longer holds f~(t-1), whatever happens below
    c->prev_valid = false;
    // on every exit: events destroyed, and (unless a best shape was
    // installed) the shape in use before the call restored
    struct Guard {
        lbm_mc_ctx* c;
        Tuning keep;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool done = false;
        ~Guard() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (!done) {
                c->tune = keep;
                const std::string msg = g_err;   // keep the failure's message
                build_tiles(c);
                g_err = msg;
            }
        }
    } guard{c, c->tune};
    HIPCHECK(hipEventCreate(&guard.e0));
    HIPCHECK(hipEventCreate(&guard.e1));
    hipEvent_t e0 = guard.e0, e1 = guard.e1;
    double best = 1e300;
    Tuning bestt = c->tune;
    for (const Tuning& t : cands) {
        if (t.split && c->hlp[0].eqb) continue;   // variant 0 only
        c->tune = t;
        lbm_mc_status st = build_tiles(c);
        if (st != LBM_MC_OK) return st;
        // a persistent grid no smaller than the tile list is the same launch
        // as the non-persistent candidate of the same shape
        if (t.persistent > 0 && t.persistent >= (int)c->htiles.size()) continue;
        for (int i = 0; i < 2; ++i) {
            st = launch_one(c, c->cur, c->prev, c->stream);
            if (st != LBM_MC_OK) return st;
        }
        HIPCHECK(hipEventRecord(e0, c->stream));
        for (int i = 0; i < reps; ++i) {
            st = launch_one(c, c->cur, c->prev, c->stream);
            if (st != LBM_MC_OK) return st;
        }
        HIPCHECK(hipEventRecord(e1, c->stream));
        HIPCHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1000.0 * ms / reps;
        if (us < best) {
            best = us;
            bestt = t;
        }
    }
    c->tune = bestt;
    lbm_mc_status st = build_tiles(c);
    if (st != LBM_MC_OK) return st;
    guard.done = true;
    if (!c->hlp[0].eqb) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const auto& q = c->params[0];
        g_tune_cache[{c->lattice, c->N, q.nx, q.ny, q.nz, c->L, tune_kind(c)}] = bestt;
    }
    if (best_us) *best_us = best;
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_set_batched_mode(lbm_mc_ctx* c, int32_t one_launch) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    c->one_launch = one_launch ? 1 : 0;
    drop_graphs(c);
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_destroy(lbm_mc_ctx* c) {
    if (!c) return LBM_MC_OK;
    if (c->stream || c->dlp) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    (void)hipFree(c->dlp);
    (void)hipFree(c->dflag);
    (void)hipFree(c->dtiles);
    (void)hipFree(c->dpartial);
    (void)hipFree(c->dtotals);
    (void)hipFree(c->dens);
    (void)hipFree(c->dmu);
    (void)hipFree(c->dgpart);
    (void)hipFree(c->dlam);
    (void)hipFree(c->dx0);
    (void)hipFree(c->adj_tiles);
    (void)hipFree(c->dprof);
    delete c;
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_adjoint_step(lbm_mc_ctx* c, const float* f_prev, const float* lam_in,
                                  float* lam_out, double* grad) {
    lbm_mc_status st = adjoint_prepare(c);
    if (st != LBM_MC_OK) return st;
    if (!f_prev || !lam_in || !lam_out || !grad)
        return fail(LBM_MC_ERR_INVALID, "adjoint_step: NULL buffer");
    if (lam_out == lam_in || lam_out == f_prev)
        return fail(LBM_MC_ERR_INVALID, "adjoint_step: lam_out must not alias lam_in or f_prev");
    const int nt = c->adj_ntiles;
    st = grad_clear(c, nt);
    if (st == LBM_MC_OK) st = adjoint_one(c, f_prev, lam_in, lam_out, c->stream);
    if (st == LBM_MC_OK) st = grad_sum(c, nt, grad);
    return st;
}

lbm_mc_status lbm_mc_adjoint_init(lbm_mc_ctx* c, const float* lam0, double* grad) {
    lbm_mc_status st = adjoint_prepare(c);
    if (st != LBM_MC_OK) return st;
    if (!lam0 || !grad) return fail(LBM_MC_ERR_INVALID, "adjoint_init: NULL buffer");
    const int nb = init_blocks(c);
    st = grad_clear(c, nb);
    if (st != LBM_MC_OK) return st;
    HIPCHECK(launch_adjoint_init(c->lattice, c->N, c->dlp, c->hlp[0], c->dx0, lam0, c->dgpart, nb,
                                 c->stream));
    return grad_sum(c, nb, grad);
}

lbm_mc_status lbm_mc_profile(lbm_mc_ctx* c, const float* state, double* xbar) {
    lbm_mc_status st = profile_check(c, state, xbar);
    if (st != LBM_MC_OK) return st;
    int rows_per, nchunks;
    profile_chunks(c, rows_per, nchunks);
    const size_t need = (size_t)nchunks * c->N * c->params[0].nx;
    if (need > c->dprof_cap) {
        if (c->dprof) (void)hipFree(c->dprof);
        c->dprof = nullptr;
        c->dprof_cap = 0;
        HIPCHECK(hipMalloc(&c->dprof, need * sizeof(double)));
        c->dprof_cap = need;
    }
    HIPCHECK(launch_profile(c->lattice, c->N, c->dlp, c->hlp[0], state, rows_per, nchunks,
                            c->dprof, xbar, c->stream));
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_profile_static(lbm_mc_ctx* c, const float* state, double* xbar) {
    lbm_mc_status st = profile_check(c, state, xbar);
    if (st != LBM_MC_OK) return st;
    const int64_t per_chunk = (int64_t)c->N * c->params[0].nx;
    if (per_chunk > kProfileScratchDoubles)
        return fail(LBM_MC_ERR_INVALID,
                    "profile_static: N * nx = %lld exceeds the fixed scratch of %lld doubles",
                    (long long)per_chunk, (long long)kProfileScratchDoubles);
    // the same row chunks as lbm_mc_profile (bit-identical results) unless
    // they do not fit the array, then fewer, longer chunks
    int rows_per, nchunks;
    profile_chunks(c, rows_per, nchunks);
    if ((int64_t)nchunks * per_chunk > kProfileScratchDoubles) {
        const int64_t rows = (int64_t)c->params[0].ny * c->params[0].nz;
        const int64_t cap = kProfileScratchDoubles / per_chunk;
        rows_per = (int)((rows + cap - 1) / cap);
        nchunks = (int)((rows + rows_per - 1) / rows_per);
    }
    HIPCHECK(launch_profile(c->lattice, c->N, c->dlp, c->hlp[0], state, rows_per, nchunks,
                            c->static_scratch, xbar, c->stream));
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_profile_vjp(lbm_mc_ctx* c, const float* state, const double* dxbar,
                                 float* lam) {
    lbm_mc_status st = profile_check(c, state, lam);
    if (st != LBM_MC_OK) return st;
    if (!dxbar) return fail(LBM_MC_ERR_INVALID, "profile_vjp: NULL buffer");
    if ((const void*)lam == (const void*)state)
        return fail(LBM_MC_ERR_INVALID, "profile_vjp: lam must not alias state");
    HIPCHECK(launch_profile_vjp(c->lattice, c->N, c->dlp, c->hlp[0], state, dxbar, lam,
                                c->cus * 8, c->stream));
    return LBM_MC_OK;
}

lbm_mc_status lbm_mc_replay(lbm_mc_ctx* c, const float* src, int64_t n, float* states,
                            int64_t stride) {
    if (!c) return fail(LBM_MC_ERR_INVALID, "ctx is NULL");
    if (!src || (!states && n > 0)) return fail(LBM_MC_ERR_INVALID, "replay: NULL buffer");
    if (n < 0) return fail(LBM_MC_ERR_INVALID, "replay: n must be >= 0");
    lbm_mc_status st = check_sequence(c, states, n, stride);
    if (st != LBM_MC_OK) return st;
    for (int64_t k = 0; k < n; ++k)
        if (states + k * stride == src)
            return fail(LBM_MC_ERR_INVALID, "replay: src is slot %lld", (long long)k);
    if (n == 0) return LBM_MC_OK;
    return run_sequence(c, 0, src, states, nullptr, n, stride, [&](hipStream_t strm) {
        const float* s = src;
        for (int64_t k = 0; k < n; ++k) {
            float* d = states + k * stride;
            lbm_mc_status r = launch_one(c, s, d, strm);
            if (r != LBM_MC_OK) return r;
            s = d;
        }
        return LBM_MC_OK;
    });
}

lbm_mc_status lbm_mc_adjoint_run(lbm_mc_ctx* c, const float* states, int64_t stride, int64_t n,
                                 const float* lam_in, float* lam_out, double* grad) {
    lbm_mc_status st = adjoint_prepare(c);
    if (st != LBM_MC_OK) return st;
    if (!states || !lam_in || !lam_out || !grad)
        return fail(LBM_MC_ERR_INVALID, "adjoint_run: NULL buffer");
    if (n < 1) return fail(LBM_MC_ERR_INVALID, "adjoint_run: n must be >= 1");
    if (lam_out == lam_in) return fail(LBM_MC_ERR_INVALID, "adjoint_run: lam_out aliases lam_in");
    st = check_sequence(c, states, n, stride);
    if (st != LBM_MC_OK) return st;
    if (n > 1 && !c->dlam) {
        HIPCHECK(hipMalloc(&c->dlam, (size_t)c->layout.total * sizeof(float)));
        HIPCHECK(hipMemsetAsync(c->dlam, 0, (size_t)c->layout.total * sizeof(float), c->stream));
    }
    const int nt = c->adj_ntiles;
    st = grad_clear(c, nt);
    if (st != LBM_MC_OK) return st;
    // kernel A of the last step, then one fused pass per earlier step (kernel
    // B of the step after it with kernel A), mu alternating between the
    // context's two buffers, and kernel B of the first step
    st = run_sequence(c, 1, states, lam_in, lam_out, n, stride, [&](hipStream_t strm) {
        const int ng = c->N * (c->N - 1) / 2 + 3;
        float* mu[2] = {c->dmu, c->dlam};
        Launch L = adjoint_launch(c, states + (n - 1) * stride, strm);
        HIPCHECK(launch_adjoint(c->lattice, c->N, L, lam_in, mu[0], c->dgpart, ng));
        for (int64_t k = 2; k <= n; ++k) {
            L = adjoint_launch(c, states + (n - k) * stride, strm);
            HIPCHECK(launch_adjoint_fused(c->lattice, c->N, L, mu[k % 2], mu[(k - 1) % 2],
                                          c->dgpart));
        }
        HIPCHECK(launch_adjoint_stream(c->lattice, c->N, L, mu[(n - 1) % 2], lam_out));
        return LBM_MC_OK;
    });
    if (st != LBM_MC_OK) return st;
    return grad_sum(c, nt, grad);
}

}  // extern "C"
