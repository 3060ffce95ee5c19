// hefk_grad.hip -- pathwise (fixed start, fixed noise) gradient of
// J = sum_s gL_s L_s (+ sum_s gL2_s L2_s, L2 = ln <w^2>) with respect to the
// trial parameters (alpha, beta):
// one thread per walker walks the checkpoint segments backwards, recomputes
// each segment from its checkpoint into a scratch tape (noise regenerated
// from Philox), and runs the adjoint recursion of hefk_adjoint.hpp over it.
// With a checkpoint at every step the stored trajectory is read directly and
// nothing is recomputed (binary64 trajectories of 2^18 walkers x 1000 steps
// take 14.7 GB of device memory).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <cmath>

#include "he_fk.h"
#include "hefk_adjoint.hpp"
#include "hefk_layout.hpp"
#include "hefk_reduce.hpp"
#include "hefk_sweep.hpp"

namespace hefk {

int check_params(const he_fk_params* p);  // hefk_kernels.hip

namespace {

constexpr int kGradBlock = layout::kLanes;
// Minimum resident waves per SIMD the gradient kernel is compiled for (register budget 512 / waves):
// 3 keeps the recomputing sweep free of spills (4 spills 164 B per lane and is no faster)
#ifndef HEFK_GRAD_WAVES
#define HEFK_GRAD_WAVES 3
#endif
#ifndef HEFK_GRAD_DIRECT_WAVES
#define HEFK_GRAD_DIRECT_WAVES 3
#endif

struct GArgs {
    TrialParams<double> tp;
    StepConst sc;
    StepScale<double> ss;
    uint32_t key0, key1;
    uint64_t walker_offset;
    int64_t n;
    int32_t n_steps, sample_every, ckpt_every, score;
    const double* ckpt;     // [n_ckpt][7][n]
    const double* samples;  // [n_samples][8]
    const double* g;        // [n_samples] weights on L_s
    const double* g2;       // [n_samples] weights on L2_s, or null
    double* tape;           // [ckpt_every + 1][7][n]
    double* partial;        // [gridDim.x][2]
    double inv_n_total, g_sum;
};

// Tape in device memory, structure of arrays over walkers (coalesced).
struct DeviceTape {
    const double* ckpt;
    double* tape;
    int64_t n, i;
    __device__ void load_ckpt(int c, double y[6], double& lnw) const
    {
        const double* b = ckpt + layout::ckpt_row(c, n);
#pragma unroll
        for (int k = 0; k < 6; ++k) y[k] = b[layout::coord(k, n, i)];
        lnw = b[layout::coord(6, n, i)];
    }
    __device__ void put(int slot, const double y[6])
    {
        double* b = tape + layout::ckpt_row(slot, n);
#pragma unroll
        for (int k = 0; k < 6; ++k) b[layout::coord(k, n, i)] = y[k];
    }
    __device__ void put_lnw(int slot, double lnw) { tape[layout::ckpt_row(slot, n) + layout::coord(6, n, i)] = lnw; }
    __device__ void get(int slot, double y[6]) const
    {
        const double* b = tape + layout::ckpt_row(slot, n);
#pragma unroll
        for (int k = 0; k < 6; ++k) y[k] = b[layout::coord(k, n, i)];
    }
    __device__ double get_lnw(int slot) const { return tape[layout::ckpt_row(slot, n) + layout::coord(6, n, i)]; }
    // the checkpoints as the stored trajectory (one per step), each read once: streaming loads
    __device__ void load_pos(int c, double y[6]) const
    {
        const double* b = ckpt + layout::ckpt_row(c, n);
#pragma unroll
        for (int k = 0; k < 6; ++k) y[k] = __builtin_nontemporal_load(b + layout::coord(k, n, i));
    }
    __device__ double load_lnw(int c) const { return ckpt[layout::ckpt_row(c, n) + layout::coord(6, n, i)]; }
};

struct SampleView {
    const double* rows;
    const double* g;
    const double* g2;
    __device__ double m(int s) const { return rows[8 * s]; }
    __device__ double s0(int s) const { return rows[8 * s + 1]; }
    __device__ double s2(int s) const { return rows[8 * s + 3]; }
    __device__ double gs(int s) const { return g[s]; }
    __device__ double g2s(int s) const { return g2 ? g2[s] : 0.0; }
};

template <int TRIAL, int NOISE, bool DIRECT>
__global__ __launch_bounds__(kGradBlock, DIRECT ? HEFK_GRAD_DIRECT_WAVES : HEFK_GRAD_WAVES) void grad_kernel(
    const GArgs a)
{
    __shared__ double red[8];
    const int64_t i = layout::walker((int64_t)blockIdx.x, threadIdx.x);
    double gth[2] = {0.0, 0.0};
    if (i < a.n) {
        const uint64_t gid = a.walker_offset + (uint64_t)i;
        Stream st;
        st.k0 = a.key0;
        st.k1 = a.key1;
        st.g0 = (uint32_t)gid;
        st.g1 = (uint32_t)(gid >> 32);
        DeviceTape tape{a.ckpt, a.tape, a.n, i};
        SampleView sv{a.samples, a.g, a.g2};
        double P = 0.0, Q = 0.0;
        if constexpr (DIRECT)
            walker_reverse_direct<TRIAL>(a.tp, a.sc, a.ss, a.n_steps, a.sample_every, sv, tape, gth, &P, &Q);
        else
            walker_reverse<TRIAL, NOISE>(a.tp, a.sc, a.ss, st, a.n_steps, a.sample_every, a.ckpt_every, sv,
                                         tape, gth, &P, &Q);
        if (a.score) {
            double y0[6], l0, sc[2];
            tape.load_ckpt(0, y0, l0);
            dlnpsi_dtheta<TRIAL>(a.tp, y0, sc);
            // start-law weight: sum_s (g_s p_is + g2_s q_is) - (sum_s g_s + g2_s) / N
            const double wgt = (P - Q) - a.g_sum * a.inv_n_total;
            gth[0] += 2.0 * sc[0] * wgt;
            gth[1] += 2.0 * sc[1] * wgt;
        }
    }
    // deterministic block sum of the two components
    const double s0 = wave_sum(gth[0]);
    const double s1 = wave_sum(gth[1]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * wave] = s0;
        red[2 * wave + 1] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = (red[0] + red[2]) + (red[4] + red[6]);
        a.partial[2 * blockIdx.x + 1] = (red[1] + red[3]) + (red[5] + red[7]);
    }
}

// Sum of the per-block partials in a fixed order (one block).
__global__ __launch_bounds__(kGradBlock) void grad_sum_kernel(const double* __restrict__ partial, int n_parts,
                                                              double* __restrict__ out)
{
    __shared__ double sh[2 * kGradBlock];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < n_parts; b += kGradBlock) {
        s0 += partial[2 * b];
        s1 += partial[2 * b + 1];
    }
    sh[2 * threadIdx.x] = s0;
    sh[2 * threadIdx.x + 1] = s1;
    __syncthreads();
    for (int w = kGradBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sh[2 * threadIdx.x] += sh[2 * (threadIdx.x + w)];
            sh[2 * threadIdx.x + 1] += sh[2 * (threadIdx.x + w) + 1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0];
        out[1] = sh[1];
    }
}

typedef void (*GradFn)(GArgs);

// the direct sweep regenerates no noise: one kernel per trial serves every noise kind
GradFn pick(int trial, int noise, bool direct)
{
    if (trial == TRIAL_EXPO) {
        if (direct) return grad_kernel<TRIAL_EXPO, NOISE_G1, true>;
        if (noise == NOISE_G1) return grad_kernel<TRIAL_EXPO, NOISE_G1, false>;
        if (noise == NOISE_G2) return grad_kernel<TRIAL_EXPO, NOISE_G2, false>;
        return grad_kernel<TRIAL_EXPO, NOISE_PM1, false>;
    }
    if (direct) return grad_kernel<TRIAL_PADE, NOISE_G1, true>;
    if (noise == NOISE_G1) return grad_kernel<TRIAL_PADE, NOISE_G1, false>;
    if (noise == NOISE_G2) return grad_kernel<TRIAL_PADE, NOISE_G2, false>;
    return grad_kernel<TRIAL_PADE, NOISE_PM1, false>;
}

struct Layout {
    size_t tape, partial, g, total;
    int64_t blocks;
};

int grad_layout(const he_fk_params* p, int64_t n_steps, int32_t sample_every, int32_t ckpt_every, Layout* L)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (p->trial != HE_FK_TRIAL_EXPO && p->trial != HE_FK_TRIAL_PADE) return HE_FK_EINVAL;
    if (p->precision != HE_FK_FP64 || p->drift_limit != 0.0 || p->flags != 0) return HE_FK_EINVAL;
    if (n_steps < 1 || sample_every < 1 || ckpt_every < 1) return HE_FK_EINVAL;
    if (n_steps % sample_every || n_steps % ckpt_every) return HE_FK_EINVAL;
    if (ckpt_every % sample_every && sample_every % ckpt_every) return HE_FK_EINVAL;
    if (n_steps >= (int64_t(1) << 31)) return HE_FK_EINVAL;
    const int64_t n = p->n_walkers;
    L->blocks = (n + kGradBlock - 1) / kGradBlock;
    if (L->blocks > INT32_MAX) return HE_FK_EINVAL;
    auto up256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    L->tape = 0;
    // the recomputing sweep's segment tape; the direct sweep (ckpt_every = 1) needs none
    L->partial = ckpt_every == 1 ? 0 : up256((size_t)(ckpt_every + 1) * 7 * (size_t)n * sizeof(double));
    L->g = L->partial + up256((size_t)L->blocks * 2 * sizeof(double));
    L->total = L->g + up256((size_t)2 * (n_steps / sample_every + 1) * sizeof(double));
    return HE_FK_OK;
}

}  // namespace
}  // namespace hefk

using namespace hefk;

extern "C" size_t he_fk_grad_scratch_bytes(const he_fk_params* p, int64_t n_steps, int32_t sample_every,
                                           int32_t ckpt_every)
{
    Layout L;
    if (grad_layout(p, n_steps, sample_every, ckpt_every, &L)) return 0;
    return L.total;
}

extern "C" int he_fk_grad(const he_fk_params* p, const double* ckpt, const double* samples, const double* gL,
                          int64_t n_steps, int32_t sample_every, int32_t ckpt_every, int32_t flags, void* scratch,
                          size_t scratch_bytes, double* dtheta, void* stream)
{
    Layout L;
    int rc = grad_layout(p, n_steps, sample_every, ckpt_every, &L);
    if (rc) return rc;
    if (!ckpt || !samples || !gL || !scratch || !dtheta) return HE_FK_EINVAL;
    if (flags & ~(HE_FK_GRAD_SCORE | HE_FK_GRAD_MOMENT2)) return HE_FK_EINVAL;
    if (scratch_bytes < L.total) return HE_FK_ESCRATCH;
    const int64_t n_samples = n_steps / sample_every + 1;
    const int64_t n_g = (flags & HE_FK_GRAD_MOMENT2) ? 2 * n_samples : n_samples;
    double g_sum = 0.0;
    for (int64_t s = 0; s < n_g; ++s) {
        if (!std::isfinite(gL[s])) return HE_FK_EINVAL;
        g_sum += gL[s];
    }
    char* base = (char*)scratch;
    GArgs a;
    memset(&a, 0, sizeof(a));
    a.tp.A = p->theta[0];
    a.tp.beta = p->theta[1];
    a.tp.c = p->theta[2];
    a.tp.a = p->theta[3];
    a.tp.Z = p->Z;
    a.tp.ee = (double)p->ee;
    a.tp.sym = 1.0;
    a.tp.r0 = 0.0;
    a.sc = make_step_const(p->dt, p->e_ref, p->quad == HE_FK_QUAD_RIGHT, 0.0, false, false);
    a.ss = step_scale(p->dt, 0.0, 0.0);
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.walker_offset = p->walker_offset;
    a.n = p->n_walkers;
    a.n_steps = (int32_t)n_steps;
    a.sample_every = sample_every;
    a.ckpt_every = ckpt_every;
    a.score = (flags & HE_FK_GRAD_SCORE) ? 1 : 0;
    a.ckpt = ckpt;
    a.samples = samples;
    a.tape = (double*)(base + L.tape);
    a.partial = (double*)(base + L.partial);
    a.g = (double*)(base + L.g);
    a.g2 = (flags & HE_FK_GRAD_MOMENT2) ? a.g + n_samples : nullptr;
    a.g_sum = g_sum;
    // 1/N of the space average: every walker of the propagate call counts (n_total of row 0)
    a.inv_n_total = 1.0 / (double)p->n_walkers;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync((void*)a.g, gL, (size_t)n_g * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return HE_FK_EDEVICE;
    const int nk = p->noise == HE_FK_NOISE_PM1 ? NOISE_PM1 : (p->contract == 2 ? NOISE_G2 : NOISE_G1);
    hipLaunchKernelGGL(pick(p->trial, nk, ckpt_every == 1), dim3((unsigned)L.blocks), dim3(kGradBlock), 0, s, a);
    if (hipGetLastError() != hipSuccess) return HE_FK_EDEVICE;
    hipLaunchKernelGGL(grad_sum_kernel, dim3(1), dim3(kGradBlock), 0, s, (const double*)a.partial, (int)L.blocks,
                       dtheta);
    return hipGetLastError() == hipSuccess ? HE_FK_OK : HE_FK_EDEVICE;
}
