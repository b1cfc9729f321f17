// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fastpi {

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// 1/sqrt(x) from the hardware estimate (relative error ~2^-24) with one third-order
// correction y (1 + e/2 + 3e^2/8), e = 1 - x y^2: error O(e^3), to FP64 rounding (normal range), in four
// dependent operations instead of the eight of two Newton steps.
__device__ __forceinline__ double rsq3(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-(x * y), y, 1.0);
    const double p = fma(0.375, e, 0.5);
    return fma(y * e, p, y);
}

// Pair `pr` of round `round` of the circle-method round robin over `qe` (even) items:
// every unordered pair appears once in qe-1 rounds and the pairs of a round are disjoint.
__host__ __device__ __forceinline__ void round_robin_pair(int round, int pr, int qe, int& a, int& b) {
    if (pr == 0) {
        a = qe - 1;
        b = round;
    } else {
        const int mod = qe - 1;
        a = (round + pr) % mod;
        b = (round - pr + mod) % mod;
    }
    if (a > b) {
        int t = a;
        a = b;
        b = t;
    }
}

// The inverse: the pair `pr` of round `round` (0 <= round < qe - 1) that holds item x, and
// x's partner in it.
__host__ __device__ __forceinline__ void round_robin_find(int round, int x, int qe, int& pr, int& other) {
    const int mod = qe - 1;
    if (x == mod || x == round) {
        pr = 0;
        other = x == mod ? round : mod;
        return;
    }
    const int d = (x - round + mod) % mod;   // x = round + d (mod qe - 1), 1 <= d < qe - 1
    if (d <= (mod - 1) / 2) {
        pr = d;
        other = (round - d + mod) % mod;
    } else {
        pr = mod - d;
        other = (round + pr) % mod;
    }
}

// Plane rotation that makes the 2x2 symmetric matrix [[app, apq], [apq, aqq]] diagonal:
// t = tan(theta) is the smaller root (Rutishauser), c = cos, s = sin. Used both for the
// one-sided (Hestenes) step, where app, aqq, apq are column inner products, and for the
// two-sided step on a symmetric matrix.
template <typename T>
__device__ __forceinline__ void jacobi_rotation(T app, T aqq, T apq, T& c, T& s, T& t) {
    const T zeta = (aqq - app) / (T(2) * apq);
    const T az = zeta < T(0) ? -zeta : zeta;
    T root;
    if (az > T(1e15)) {
        root = az;   // sqrt(1 + zeta^2) ~ |zeta|; avoids overflow of zeta^2
    } else {
        root = sqrt(T(1) + zeta * zeta);
    }
    t = T(1) / (az + root);
    if (zeta < T(0)) t = -t;
    c = T(1) / sqrt(T(1) + t * t);
    s = c * t;
}

}  // namespace fastpi
