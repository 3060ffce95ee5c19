// hefk_kernels.hip -- gfx950 kernels and the C ABI entry points of libhefk
// (start ensemble, persistent walker propagation with a log-domain space
// average at sampling times, deterministic merge of block partials).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <cmath>
#include <mutex>

#include "he_fk.h"
#include "hefk_device.hpp"
#include "hefk_layout.hpp"
#include "hefk_reduce.hpp"

namespace hefk {

constexpr int kBlock = layout::kLanes;  // 4 waves of 64 lanes; one walker per lane

// Minimum resident waves per SIMD the propagate kernels are compiled for
// (register budget 512 / waves: 80 registers in binary32, 128 in binary64).  At these
// budgets the step loops with Gaussian increments have no spills, and those of the +-1
// walk keep at most two scratch accesses per step; the other spills are in the sampling
// code, run once per sampling interval.
#ifndef HEFK_WAVES_F32
#define HEFK_WAVES_F32 6
#endif
#ifndef HEFK_WAVES_F64
#define HEFK_WAVES_F64 4
#endif
// The kernels with the variant flags (plain walk, node bridge) carry both variants'
// code in their step loop.  For the trial functions with an angular factor or a
// second orbital that loop spills at the budgets above, and fewer, wider waves win.
#ifndef HEFK_WAVES_F32_EXT
#define HEFK_WAVES_F32_EXT 4
#endif
#ifndef HEFK_WAVES_F64_EXT
#define HEFK_WAVES_F64_EXT 3
#endif

template <typename R, int TRIAL, bool EXT>
constexpr int propagate_waves()
{
    constexpr bool heavy = EXT && TRIAL != TRIAL_EXPO && TRIAL != TRIAL_PADE;
    if (sizeof(R) == 4) return heavy ? HEFK_WAVES_F32_EXT : HEFK_WAVES_F32;
    return heavy ? HEFK_WAVES_F64_EXT : HEFK_WAVES_F64;
}

struct KArgs {
    TrialParams<double> tpd;
    TrialParams<float> tpf;
    StepConst sc;
    StepScale<double> ssd;
    StepScale<float> ssf;
    double init_sigma, metropolis_sigma;
    uint32_t key0, key1;
    uint64_t walker_offset;
    int64_t n;
    int32_t n_metropolis;
    int32_t step0, n_steps, sample_every, n_samples, ckpt_every;
    int32_t rows_in_lds;  // the block's partial rows accumulate in LDS, written to `partials` once
    void* x;
    double* lnw;
    void* el;
    double* partials;  // [gridDim.x][n_samples][8]
    double* ckpt;      // [n_ckpt][7][n] or null
};

template <typename R>
__device__ __forceinline__ const TrialParams<R>& tparams(const KArgs& a);
template <>
__device__ __forceinline__ const TrialParams<double>& tparams<double>(const KArgs& a)
{
    return a.tpd;
}
template <>
__device__ __forceinline__ const TrialParams<float>& tparams<float>(const KArgs& a)
{
    return a.tpf;
}

template <typename R>
__device__ __forceinline__ const StepScale<R>& sscale(const KArgs& a);
template <>
__device__ __forceinline__ const StepScale<double>& sscale<double>(const KArgs& a)
{
    return a.ssd;
}
template <>
__device__ __forceinline__ const StepScale<float>& sscale<float>(const KArgs& a)
{
    return a.ssf;
}

__device__ __forceinline__ Stream make_stream(const KArgs& a, int64_t i)
{
    const uint64_t g = a.walker_offset + (uint64_t)i;
    Stream s;
    s.k0 = a.key0;
    s.k1 = a.key1;
    s.g0 = (uint32_t)g;
    s.g1 = (uint32_t)(g >> 32);
    return s;
}

// ---------------------------------------------------------------------------
// Start ensemble: Gaussian draw, Metropolis on |psi|^2 (binary64), then the
// local energy at the stored (possibly binary32) position.
// ---------------------------------------------------------------------------
template <typename R, int TRIAL>
__global__ __launch_bounds__(kBlock) void init_kernel(const KArgs a)
{
    const int64_t i = layout::walker((int64_t)blockIdx.x, threadIdx.x);
    if (i >= a.n) return;
    const Stream st = make_stream(a, i);
    double y[6];
    init_walker<TRIAL>(a.tpd, st, a.n_metropolis, a.init_sigma, a.metropolis_sigma, y);
    R yr[6], b[6], el;
#pragma unroll
    for (int k = 0; k < 6; ++k) yr[k] = (R)y[k];
    trial_eval<R, TRIAL>(tparams<R>(a), yr, b, el);
    R* x = (R*)a.x;
#pragma unroll
    for (int k = 0; k < 6; ++k) x[layout::coord(k, a.n, i)] = yr[k];
    ((R*)a.el)[i] = el;
    a.lnw[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Persistent propagation.  Each block walks over chunks of 256 walkers
// (chunk c = blockIdx.x + j * gridDim.x); each lane keeps its walker in
// registers for all n_steps steps.  At every sampling time the block reduces
// (max ln w, then S0, S1, S2 and counts) and merges the result into its own
// partial row.  The rows accumulate in LDS when they fit (kRowsLdsBytes) and
// go to the workspace once, at the end; otherwise they are merged in place in
// the workspace, chunk after chunk.
// ---------------------------------------------------------------------------
#ifndef HEFK_ROWS_LDS_BYTES
#define HEFK_ROWS_LDS_BYTES 16384  // 256 sample rows of 64 bytes per block (0: rows merged in the workspace)
#endif
constexpr int kRowsLdsBytes = HEFK_ROWS_LDS_BYTES;
template <typename R, bool OWN_EXP>
__device__ __forceinline__ void sample_row(const KArgs& a, int row, double* rows_out, double* rows_lds, bool first,
                                           bool valid, const WalkerState<R>& w, double* red)
{
    Tuple t = block_tuple<OWN_EXP>(valid, w.lnw, (double)w.el, red);
    if (threadIdx.x == 0) {
        // two paths, so that each row access has a known address space (LDS or global)
        if (a.rows_in_lds) {
            double* r = rows_lds + layout::row_offset(row);
            if (!first) t = merge_tuple(load_tuple(r), t);
            store_tuple(r, t);
        } else {
            double* r = rows_out + layout::row_offset(row);
            if (!first) t = merge_tuple(load_tuple(r), t);
            store_tuple(r, t);
        }
    }
}

template <typename R, int TRIAL, int NOISE, bool EXT>
__global__ __launch_bounds__(kBlock, (propagate_waves<R, TRIAL, EXT>())) void propagate_kernel(
    const KArgs a)
{
    // the binary64 variant kernels (plain walk, node bridge) of the two-orbital trials take
    // the sample weights by the step's own exp: the library's spilled part of their step
    // loop to scratch (measured: P_z with the bridge 3.5 % and fn 7 with bridge and plain walk
    // 9 % faster without it; the other kernels measured the same or faster as they are)
    constexpr bool kOwnExp = sizeof(R) == 8 && EXT && TRIAL != TRIAL_EXPO && TRIAL != TRIAL_PADE;
    __shared__ double red[kRedSlots];
    extern __shared__ double rows_lds[];  // [n_samples][8] when a.rows_in_lds
    const TrialParams<R>& tp = tparams<R>(a);
    const StepScale<R>& ss = sscale<R>(a);
    const int64_t n = a.n;
    const int64_t n_chunks = layout::chunks(n);
    double* const rows_out = a.partials + HEFK_BLOCK_ROWS(blockIdx.x, a.n_samples);
    R* x = (R*)a.x;

    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const bool first = (c == (int64_t)blockIdx.x);
        const int64_t i = layout::walker(c, threadIdx.x);
        const bool valid = i < n;
        const int64_t ii = valid ? i : n - 1;  // tail lanes shadow the last walker, never stored or counted
        const Stream st = make_stream(a, ii);
        WalkerState<R> w;
#pragma unroll
        for (int k = 0; k < 6; ++k) w.y[k] = x[layout::coord(k, n, ii)];
        w.lnw = a.lnw[ii];
        walker_reset<R, TRIAL, EXT>(tp, a.sc, ss, w);

        sample_row<R, kOwnExp>(a, 0, rows_out, rows_lds, first, valid, w, red);
        if (a.ckpt && valid) {
#pragma unroll
            for (int k = 0; k < 6; ++k) a.ckpt[layout::coord(k, n, i)] = (double)w.y[k];
            a.ckpt[layout::coord(6, n, i)] = w.lnw;
        }

        int row = 1, until_sample = a.sample_every, until_ckpt = a.ckpt_every, crow = 1;
        NoiseGen<R, NOISE> noise;
        for (int k = 0; k < a.n_steps; ++k) {
            Increment<R> inc;
            noise.draw(st, (uint32_t)(a.step0 + k), ss, inc);
            walker_step<R, TRIAL, EXT>(tp, a.sc, ss, inc, w);
            if (--until_sample == 0) {
                until_sample = a.sample_every;
                sample_row<R, kOwnExp>(a, row, rows_out, rows_lds, first, valid, w, red);
                ++row;
            }
            if (a.ckpt && --until_ckpt == 0) {
                until_ckpt = a.ckpt_every;
                if (valid) {
                    double* cp = a.ckpt + layout::ckpt_row(crow, n);
                    // streaming stores: a checkpoint is written once and read once, by the
                    // gradient's reverse sweep, long after (a trajectory when ckpt_every = 1)
#pragma unroll
                    for (int kk = 0; kk < 6; ++kk)
                        __builtin_nontemporal_store((double)w.y[kk], cp + layout::coord(kk, n, i));
                    __builtin_nontemporal_store(w.lnw, cp + layout::coord(6, n, i));
                }
                ++crow;
            }
        }
        if (valid) {
#pragma unroll
            for (int k = 0; k < 6; ++k) x[layout::coord(k, n, i)] = w.y[k];
            a.lnw[i] = w.lnw;
            ((R*)a.el)[i] = w.el;
        }
    }
    if (a.rows_in_lds) {
        __syncthreads();  // thread 0's last merge into LDS is complete
        for (int k = threadIdx.x; k < a.n_samples * 8; k += kBlock) rows_out[k] = rows_lds[k];
    }
}

// Merge the per-block partial rows of one sample (blockIdx.x) in a fixed order.
__global__ __launch_bounds__(kBlock) void merge_kernel(const double* __restrict__ partials, int n_parts,
                                                       int n_samples, double* __restrict__ samples)
{
    __shared__ double sh[kBlock * 8];
    const int s = blockIdx.x;
    Tuple t = empty_tuple();
    for (int b = threadIdx.x; b < n_parts; b += kBlock)
        t = merge_tuple(t, load_tuple(partials + layout::block_rows(b, n_samples) + layout::row_offset(s)));
    store_tuple(sh + threadIdx.x * 8, t);
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            Tuple l = load_tuple(sh + threadIdx.x * 8);
            Tuple r = load_tuple(sh + (threadIdx.x + w) * 8);
            store_tuple(sh + threadIdx.x * 8, merge_tuple(l, r));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) store_tuple(samples + (size_t)s * 8, load_tuple(sh));
}

// ---------------------------------------------------------------------------
// Host side: argument checks, kernel choice, launch geometry.
// ---------------------------------------------------------------------------
typedef void (*KernelFn)(KArgs);

template <typename R, int TRIAL, bool EXT>
KernelFn pick_propagate(int noise)
{
    switch (noise) {
        case NOISE_G1: return propagate_kernel<R, TRIAL, NOISE_G1, EXT>;
        case NOISE_G2: return propagate_kernel<R, TRIAL, NOISE_G2, EXT>;
        default: return propagate_kernel<R, TRIAL, NOISE_PM1, EXT>;
    }
}

template <typename R, bool EXT>
KernelFn pick_propagate_t(int trial, int noise)
{
    switch (trial) {
        case TRIAL_EXPO: return pick_propagate<R, TRIAL_EXPO, EXT>(noise);
        case TRIAL_PADE: return pick_propagate<R, TRIAL_PADE, EXT>(noise);
        case TRIAL_TRIPLET: return pick_propagate<R, TRIAL_TRIPLET, EXT>(noise);
        case TRIAL_TRIPLET_R0: return pick_propagate<R, TRIAL_TRIPLET_R0, EXT>(noise);
        case TRIAL_PZ_SUM: return pick_propagate<R, TRIAL_PZ_SUM, EXT>(noise);
        default: return pick_propagate<R, TRIAL_PZ, EXT>(noise);
    }
}

// The generalized walk without variants runs kernels that carry no flag tests.
template <typename R>
KernelFn pick_propagate_r(int trial, int noise, int flags)
{
    return flags ? pick_propagate_t<R, true>(trial, noise) : pick_propagate_t<R, false>(trial, noise);
}

template <typename R>
KernelFn pick_init_r(int trial)
{
    switch (trial) {
        case TRIAL_EXPO: return init_kernel<R, TRIAL_EXPO>;
        case TRIAL_PADE: return init_kernel<R, TRIAL_PADE>;
        case TRIAL_TRIPLET: return init_kernel<R, TRIAL_TRIPLET>;
        case TRIAL_TRIPLET_R0: return init_kernel<R, TRIAL_TRIPLET_R0>;
        case TRIAL_PZ_SUM: return init_kernel<R, TRIAL_PZ_SUM>;
        default: return init_kernel<R, TRIAL_PZ>;
    }
}

static int noise_kind(const he_fk_params* p)
{
    if (p->noise == HE_FK_NOISE_PM1) return NOISE_PM1;
    return p->contract == 2 ? NOISE_G2 : NOISE_G1;
}

static KernelFn propagate_fn(const he_fk_params* p)
{
    return p->precision == HE_FK_MIXED ? pick_propagate_r<float>(p->trial, noise_kind(p), p->flags)
                                       : pick_propagate_r<double>(p->trial, noise_kind(p), p->flags);
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_params(const he_fk_params* p)
{
    if (!p) return HE_FK_EINVAL;
    if (p->trial < HE_FK_TRIAL_EXPO || p->trial > HE_FK_TRIAL_PZ_SUM) return HE_FK_EINVAL;
    if (p->trial == HE_FK_TRIAL_PZ && p->sym != 1 && p->sym != -1) return HE_FK_EINVAL;
    if (p->ee != 0 && p->ee != 1) return HE_FK_EINVAL;
    if (p->noise != HE_FK_NOISE_GAUSS && p->noise != HE_FK_NOISE_PM1) return HE_FK_EINVAL;
    if (p->quad != HE_FK_QUAD_TRAPEZOID && p->quad != HE_FK_QUAD_RIGHT) return HE_FK_EINVAL;
    if (p->contract != 1 && p->contract != 2) return HE_FK_EINVAL;
    if (p->precision != HE_FK_FP64 && p->precision != HE_FK_MIXED) return HE_FK_EINVAL;
    if (p->n_metropolis < 0) return HE_FK_EINVAL;
    if ((p->flags & ~(HE_FK_FLAG_PLAIN | HE_FK_FLAG_BRIDGE)) || p->reserved != 0) return HE_FK_EINVAL;
    if ((p->flags & HE_FK_FLAG_PLAIN) && p->drift_limit != 0.0) return HE_FK_EINVAL;
    if ((p->flags & HE_FK_FLAG_BRIDGE) && (p->trial == HE_FK_TRIAL_EXPO || p->trial == HE_FK_TRIAL_PADE))
        return HE_FK_EINVAL;
    if (!finite_pos(p->Z) || !finite_pos(p->dt) || !finite_pos(p->metropolis_sigma) ||
        !finite_pos(p->init_sigma) || !std::isfinite(p->e_ref) || !(p->drift_limit >= 0.0) ||
        !std::isfinite(p->drift_limit))
        return HE_FK_EINVAL;
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(p->theta[k])) return HE_FK_EINVAL;
    if (!(p->theta[0] > 0.0)) return HE_FK_EINVAL;
    if (p->trial != HE_FK_TRIAL_EXPO && !(p->theta[1] >= 0.0)) return HE_FK_EINVAL;
    if (p->n_walkers < 1 || p->n_walkers > (int64_t(1) << 40)) return HE_FK_EINVAL;
    if (p->walker_offset > UINT64_MAX - (uint64_t)p->n_walkers) return HE_FK_EINVAL;
    return HE_FK_OK;
}

static KArgs make_args(const he_fk_params* p)
{
    KArgs a;
    memset(&a, 0, sizeof(a));
    a.tpd.A = p->theta[0];
    a.tpd.beta = p->theta[1];
    a.tpd.c = p->theta[2];
    a.tpd.a = p->theta[3];
    a.tpd.Z = p->Z;
    a.tpd.ee = (double)p->ee;
    a.tpd.sym = (double)(p->trial == HE_FK_TRIAL_PZ ? p->sym : 1);
    a.tpd.r0 = p->theta[4];
    a.tpf.r0 = (float)a.tpd.r0;
    a.tpf.A = (float)a.tpd.A;
    a.tpf.beta = (float)a.tpd.beta;
    a.tpf.c = (float)a.tpd.c;
    a.tpf.a = (float)a.tpd.a;
    a.tpf.Z = (float)a.tpd.Z;
    a.tpf.ee = (float)a.tpd.ee;
    a.tpf.sym = (float)a.tpd.sym;
    a.sc = make_step_const(p->dt, p->e_ref, p->quad == HE_FK_QUAD_RIGHT, p->drift_limit,
                           (p->flags & HE_FK_FLAG_PLAIN) != 0, (p->flags & HE_FK_FLAG_BRIDGE) != 0);
    a.ssd = step_scale(p->dt, p->drift_limit, 0.0);
    a.ssf = step_scale(p->dt, p->drift_limit, 0.0f);
    a.init_sigma = p->init_sigma;
    a.metropolis_sigma = p->metropolis_sigma;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.walker_offset = p->walker_offset;
    a.n = p->n_walkers;
    a.n_metropolis = p->n_metropolis;
    return a;
}

// Dynamic LDS of a propagate launch: the block's partial rows when they fit.
static size_t rows_lds_bytes(int64_t n_samples)
{
    const size_t b = layout::row_offset(n_samples) * sizeof(double);
    return b <= (size_t)kRowsLdsBytes ? b : 0;
}

// Blocks of a propagate launch: every block resident at once, none without a chunk.
static int propagate_grid(const he_fk_params* p, size_t lds_bytes, int64_t* out)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HE_FK_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return HE_FK_EDEVICE;
    KernelFn fn = propagate_fn(p);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, kBlock, lds_bytes) != hipSuccess)
        return HE_FK_EDEVICE;
    if (per_cu < 1) per_cu = 1;
    *out = layout::grid(layout::chunks(p->n_walkers), (int64_t)cus * per_cu);
    return HE_FK_OK;
}

static int check_steps(int64_t step0, int64_t n_steps, int32_t sample_every)
{
    if (step0 < 0 || n_steps < 0 || sample_every < 1) return HE_FK_EINVAL;
    if (n_steps % sample_every != 0) return HE_FK_EINVAL;
    if (step0 + n_steps >= (int64_t(1) << 31)) return HE_FK_EINVAL;
    return HE_FK_OK;
}

// Argument checks, then the propagate kernel and the merge of its per-block partial rows,
// which go to `workspace` (at least `workspace_bytes` bytes of device memory).
static int propagate_launch(const he_fk_params* p, const he_fk_walkers* w, int64_t step0, int64_t n_steps,
                            int32_t sample_every, double* samples, double* ckpt, int32_t ckpt_every,
                            void* workspace, size_t workspace_bytes, void* stream)
{
    int rc = check_params(p);
    if (rc) return rc;
    rc = check_steps(step0, n_steps, sample_every);
    if (rc) return rc;
    if (!w || !w->x || !w->lnw || !w->el || !samples || !workspace) return HE_FK_EINVAL;
    if (ckpt) {
        if (p->precision != HE_FK_FP64 || ckpt_every < 1 || n_steps % ckpt_every != 0) return HE_FK_EINVAL;
    }
    const int64_t n_samples = n_steps / sample_every + 1;
    const size_t lds = rows_lds_bytes(n_samples);
    int64_t g = 0;
    rc = propagate_grid(p, lds, &g);
    if (rc) return rc;
    const size_t need = layout::block_rows(g, n_samples) * sizeof(double);
    if (workspace_bytes < need) return HE_FK_ESCRATCH;
    KArgs a = make_args(p);
    a.x = w->x;
    a.lnw = w->lnw;
    a.el = w->el;
    a.step0 = (int32_t)step0;
    a.n_steps = (int32_t)n_steps;
    a.sample_every = sample_every;
    a.n_samples = (int32_t)n_samples;
    a.ckpt_every = ckpt ? ckpt_every : 0;
    a.ckpt = ckpt;
    a.partials = (double*)workspace;
    a.rows_in_lds = lds ? 1 : 0;
    hipLaunchKernelGGL(propagate_fn(p), dim3((unsigned)g), dim3(kBlock), lds, (hipStream_t)stream, a);
    if (hipGetLastError() != hipSuccess) return HE_FK_EDEVICE;
    hipLaunchKernelGGL(merge_kernel, dim3((unsigned)n_samples), dim3(kBlock), 0, (hipStream_t)stream,
                       (const double*)workspace, (int)g, (int)n_samples, samples);
    return hipGetLastError() == hipSuccess ? HE_FK_OK : HE_FK_EDEVICE;
}

// ---------------------------------------------------------------------------
// Scratch of he_fk_propagate_noalloc: the per-block partial rows live in this
// static device array (one copy per GPU, held until the process ends).  Every
// block writes its rows before it reads them, so nothing needs clearing.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in symbol): its device address is looked up once per device, with that
// device current, and kept here.
// ---------------------------------------------------------------------------
__device__ __align__(256) double scratch[HE_FK_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices];

static int static_scratch(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HE_FK_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return HE_FK_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HE_FK_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HE_FK_OK;
}

}  // namespace hefk

using namespace hefk;

extern "C" {

int he_fk_init(const he_fk_params* p, const he_fk_walkers* w, void* stream)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (!w || !w->x || !w->lnw || !w->el) return HE_FK_EINVAL;
    KArgs a = make_args(p);
    a.x = w->x;
    a.lnw = w->lnw;
    a.el = w->el;
    KernelFn fn = p->precision == HE_FK_MIXED ? pick_init_r<float>(p->trial) : pick_init_r<double>(p->trial);
    const int64_t blocks = layout::chunks(p->n_walkers);
    if (blocks > INT32_MAX) return HE_FK_EINVAL;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? HE_FK_OK : HE_FK_EDEVICE;
}

size_t he_fk_propagate_workspace_bytes(const he_fk_params* p, int64_t n_steps, int32_t sample_every)
{
    if (check_params(p) || check_steps(0, n_steps, sample_every)) return 0;
    const int64_t n_samples = n_steps / sample_every + 1;
    int64_t g = 0;
    if (propagate_grid(p, rows_lds_bytes(n_samples), &g)) return 0;
    return layout::block_rows(g, n_samples) * sizeof(double);
}

int he_fk_propagate(const he_fk_params* p, const he_fk_walkers* w, int64_t step0, int64_t n_steps,
                    int32_t sample_every, double* samples, double* ckpt, int32_t ckpt_every, void* workspace,
                    size_t workspace_bytes, void* stream)
{
    if (!workspace) return HE_FK_EINVAL;
    return propagate_launch(p, w, step0, n_steps, sample_every, samples, ckpt, ckpt_every, workspace,
                            workspace_bytes, stream);
}

int he_fk_propagate_noalloc(const he_fk_params* p, const he_fk_walkers* w, int64_t step0, int64_t n_steps,
                            int32_t sample_every, double* samples, double* ckpt, int32_t ckpt_every, void* stream)
{
    int rc = check_params(p);
    if (rc) return rc;
    rc = check_steps(step0, n_steps, sample_every);
    if (rc) return rc;
    void* ws = nullptr;
    rc = static_scratch(&ws);
    if (rc) return rc;
    return propagate_launch(p, w, step0, n_steps, sample_every, samples, ckpt, ckpt_every, ws,
                            (size_t)HE_FK_NOALLOC_SCRATCH_BYTES, stream);
}
const char* he_fk_strerror(int code)
{
    switch (code) {
        case HE_FK_OK: return "ok";
        case HE_FK_EINVAL: return "invalid argument";
        case HE_FK_EDEVICE: return "HIP device error";
        case HE_FK_ENONFINITE: return "non-finite ln w or local energy in a sample row";
        case HE_FK_EALLDEAD: return "no live walker in a sample row";
        case HE_FK_ESCRATCH: return "workspace or scratch too small";
        default: return "unknown error";
    }
}

}  // extern "C"
