// Compile-time velocity sets.
//
// D2Q9 uses the paper's numbering (Sec. 2, equation of the species discrete
// velocities): 0 rest, 1..4 = (1,0),(0,1),(-1,0),(0,-1), 5..8 = (1,1),(-1,1),
// (-1,-1),(1,-1).  D3Q19 (not in the paper) uses rest, the six axis
// directions and the twelve edge directions.  The species velocity is
// e^i_alpha = c_i * (cx, cy, cz)(alpha).
#pragma once

namespace lbmmc {

template <int LAT>
struct Lat;

template <>
struct Lat<0> {
    static constexpr int Q = 9;
    static constexpr int DIM = 2;
    __host__ __device__ static constexpr int cx(int a) {
        constexpr int t[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        return t[a];
    }
    __host__ __device__ static constexpr int cy(int a) {
        constexpr int t[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        return t[a];
    }
    __host__ __device__ static constexpr int cz(int) { return 0; }
    __host__ __device__ static constexpr int opp(int a) {
        constexpr int t[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        return t[a];
    }
    __host__ __device__ static constexpr float w(int a) {
        return a == 0 ? 4.0f / 9.0f : (a < 5 ? 1.0f / 9.0f : 1.0f / 36.0f);
    }
    // w_a / w_0 (exact powers of two), 1/w_0 (exact) and 1/(1 - w_0)
    __host__ __device__ static constexpr float wr(int a) {
        return a == 0 ? 1.0f : (a < 5 ? 0.25f : 0.0625f);
    }
    static constexpr float inv_w0 = 2.25f;
    static constexpr float inv_1mw0 = 1.8f;
};

template <>
struct Lat<1> {
    static constexpr int Q = 19;
    static constexpr int DIM = 3;
    __host__ __device__ static constexpr int cx(int a) {
        constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return t[a];
    }
    __host__ __device__ static constexpr int cy(int a) {
        constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
        return t[a];
    }
    __host__ __device__ static constexpr int cz(int a) {
        constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return t[a];
    }
    __host__ __device__ static constexpr int opp(int a) {
        constexpr int t[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
        return t[a];
    }
    __host__ __device__ static constexpr float w(int a) {
        return a == 0 ? 1.0f / 3.0f : (a < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
    }
    // w_a / w_0, and 1/w_0, 1/(1 - w_0)
    __host__ __device__ static constexpr float wr(int a) {
        return a == 0 ? 1.0f : (a < 7 ? 1.0f / 6.0f : 1.0f / 12.0f);
    }
    static constexpr float inv_w0 = 3.0f;
    static constexpr float inv_1mw0 = 1.5f;
};

// Components of a direction in the kernel's frame: the slowest ("march")
// axis is y in 2-D and z in 3-D; the cross-section axes are x (and y in 3-D).
template <int LAT>
struct Frame {
    using L = Lat<LAT>;
    static constexpr int DIM = L::DIM;
    static constexpr int MA = DIM - 1;  // march axis index (1 = y, 2 = z)
    __host__ __device__ static constexpr int p0(int a) { return L::cx(a); }
    __host__ __device__ static constexpr int p1(int a) { return DIM == 3 ? L::cy(a) : 0; }
    __host__ __device__ static constexpr int pm(int a) { return DIM == 3 ? L::cz(a) : L::cy(a); }
    __host__ __device__ static constexpr int comp(int a, int axis) {
        return axis == 0 ? L::cx(a) : (axis == 1 ? L::cy(a) : L::cz(a));
    }
};

}  // namespace lbmmc
