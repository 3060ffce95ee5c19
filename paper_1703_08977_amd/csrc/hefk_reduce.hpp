// hefk_reduce.hpp -- log-domain space average across walkers.
//
// A partial row over a set of walkers is the tuple
//   (m, S0, S1, S2, n_alive, n_nonfinite, n_total)
// with m = max ln w over live walkers, S0 = sum e^(ln w - m),
// S1 = sum e^(ln w - m) E_L, S2 = sum e^(2 (ln w - m)).  Two rows merge by
// rescaling to the larger maximum.  Inside a wavefront the sums and the
// maximum go through DPP lane exchanges (quad permutes, half-row and row
// mirrors) and one ds_swizzle across the two 16-lane rows of each half-wave;
// the four waves of a block meet in LDS.  Every reduction has a fixed shape,
// so results are bitwise repeatable.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "hefk_f64math.hpp"

namespace hefk {

struct Tuple {
    double m, s0, s1, s2, alive, bad, total;
};

__host__ __device__ __forceinline__ Tuple empty_tuple()
{
    Tuple t;
    t.m = -INFINITY;
    t.s0 = t.s1 = t.s2 = 0.0;
    t.alive = t.bad = t.total = 0.0;
    return t;
}

__host__ __device__ __forceinline__ Tuple merge_tuple(const Tuple& x, const Tuple& y)
{
    Tuple t;
    t.m = fmax(x.m, y.m);
    if (t.m == -INFINITY) {
        t.s0 = t.s1 = t.s2 = 0.0;
    } else {
        const double ex = exp(x.m - t.m), ey = exp(y.m - t.m);
        t.s0 = x.s0 * ex + y.s0 * ey;
        t.s1 = x.s1 * ex + y.s1 * ey;
        t.s2 = x.s2 * (ex * ex) + y.s2 * (ey * ey);
    }
    t.alive = x.alive + y.alive;
    t.bad = x.bad + y.bad;
    t.total = x.total + y.total;
    return t;
}

__host__ __device__ __forceinline__ Tuple load_tuple(const double* p)
{
    Tuple t;
    t.m = p[0];
    t.s0 = p[1];
    t.s1 = p[2];
    t.s2 = p[3];
    t.alive = p[4];
    t.bad = p[5];
    t.total = p[6];
    return t;
}

__host__ __device__ __forceinline__ void store_tuple(double* p, const Tuple& t)
{
    p[0] = t.m;
    p[1] = t.s0;
    p[2] = t.s1;
    p[3] = t.s2;
    p[4] = t.alive;
    p[5] = t.bad;
    p[6] = t.total;
    p[7] = 0.0;
}

// ---- wavefront exchanges of a binary64 value (two 32-bit DPP moves) ----
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double swz_xor16_f64(double v)
{
    // ds_swizzle bit mode: and 0x1F, or 0, xor 0x10 within each 32-lane half
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_ds_swizzle(lo, 0x401F);
    hi = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_f64(double v, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

enum : int {
    kDppXor1 = 0xB1,        // quad_perm [1,0,3,2]
    kDppXor2 = 0x4E,        // quad_perm [2,3,0,1]
    kDppHalfMirror = 0x141, // row_half_mirror: lane i <- 7 - i within 8
    kDppMirror = 0x140,     // row_mirror: lane i <- 15 - i within 16
};

// Sum over the 64 lanes; every lane gets the same bits.
__device__ __forceinline__ double wave_sum(double v)
{
    v = v + dpp_f64<kDppXor1>(v);
    v = v + dpp_f64<kDppXor2>(v);
    v = v + dpp_f64<kDppHalfMirror>(v);
    v = v + dpp_f64<kDppMirror>(v);
    v = v + swz_xor16_f64(v);
    return lane_f64(v, 0) + lane_f64(v, 32);
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_f64<kDppXor1>(v));
    v = fmax(v, dpp_f64<kDppXor2>(v));
    v = fmax(v, dpp_f64<kDppHalfMirror>(v));
    v = fmax(v, dpp_f64<kDppMirror>(v));
    v = fmax(v, swz_xor16_f64(v));
    return fmax(lane_f64(v, 0), lane_f64(v, 32));
}

constexpr int kRedSlots = 4 * 8;  // 4 waves x 8 doubles

// Block-wide tuple over the block's 256 lanes (blockDim.x == 256); the result
// is valid in thread 0.  All threads of the block must call it.  Two barriers
// per call: every thread has read the maxima red[0..3] of a call before that
// call's second barrier, and thread 0 has read its sums red[4..] before it
// reaches the next call's first barrier, which the next sums are written after;
// so consecutive calls need no barrier between them.
// OWN_EXP: the weights e^(ln w - m) by the step's own binary64 exp (hefk_f64math.hpp), in
// the binary64 kernels: the library exp needs more registers than their step loop leaves
// free and spilled part of the loop's state to scratch.
template <bool OWN_EXP = false>
__device__ __forceinline__ Tuple block_tuple(bool valid, double lnw, double el, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool bad = valid && (isnan(lnw) || lnw == INFINITY);
    const bool alive = valid && !bad && lnw != -INFINITY;
    const double lv = alive ? lnw : -INFINITY;
    const double mw = wave_max(lv);
    if (lane == 0) red[wave] = mw;
    __syncthreads();
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double e = alive ? (OWN_EXP ? f64::exp(lnw - m) : exp(lnw - m)) : 0.0;
    const double s0 = wave_sum(e);
    const double s1 = wave_sum(alive ? e * el : 0.0);
    const double s2 = wave_sum(e * e);
    const double na = (double)__popcll(__ballot(alive));
    const double nb = (double)__popcll(__ballot(bad));
    const double nt = (double)__popcll(__ballot(valid));
    if (lane == 0) {
        double* r = red + 4 + wave * 6;
        r[0] = s0;
        r[1] = s1;
        r[2] = s2;
        r[3] = na;
        r[4] = nb;
        r[5] = nt;
    }
    __syncthreads();
    Tuple t;
    t.m = m;
    t.s0 = t.s1 = t.s2 = t.alive = t.bad = t.total = 0.0;
    if (threadIdx.x == 0) {
        for (int wv = 0; wv < 4; ++wv) {
            const double* r = red + 4 + wv * 6;
            t.s0 += r[0];
            t.s1 += r[1];
            t.s2 += r[2];
            t.alive += r[3];
            t.bad += r[4];
            t.total += r[5];
        }
    }
    return t;
}

}  // namespace hefk
