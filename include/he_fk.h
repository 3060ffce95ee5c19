/*
 * he_fk.h -- C ABI of libhefk: importance-sampled (generalized) Feynman-Kac
 * propagation of two-electron (He) walkers on AMD Instinct MI355X (gfx950).
 *
 * Method (Datta, Rejcek, Fry, "The He atom revisited", arXiv:1703.08977):
 *   The lowest eigenvalue of H = -Lap/2 + V on R^6, V = -Z/r1 - Z/r2 + 1/r12,
 *   follows from eq. (4):
 *     lambda1 = lambda0 - lim_t (1/t) ln E[ exp(-int_0^t V_P(Y(s)) ds) ],
 *   with V_P = E_L - lambda0, E_L = -(1/2) Lap(psi_T)/psi_T + V the local
 *   energy of the trial function psi_T (the paper's V0 lacks the factor 1/2
 *   on Lap(phi)/phi; with it psi_T^2 is the stationary law of Y), and Y the
 *   drifted diffusion dY = grad(psi_T)/psi_T dt + dX that follows eq. (4).
 *   The expectation is a space average over independent replications
 *   (walkers), kept in the log domain: L(t) = ln( (1/N) sum_i w_i(t) ),
 *   ln w_i = -sum_k V_P dt along walker i's discretised path.  Walkers of
 *   excited-state trials are absorbed when they cross the node of psi_T.
 *
 * Conventions for every entry point:
 *   - Device pointers are caller-owned device memory; the library never
 *     allocates device memory.  Host pointers are named so in each comment.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     null stream); outputs are valid after that stream synchronises.
 *   - Return 0 on success or a negative HE_FK_E* code; nothing is enqueued
 *     when an argument check fails.  No exception crosses the ABI.  Apart from
 *     the static scratch of he_fk_propagate_noalloc, the library holds no
 *     mutable global state: calls on distinct buffers may run concurrently
 *     from different threads.
 */
#ifndef HE_FK_H
#define HE_FK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define HE_FK_OK 0
#define HE_FK_EINVAL (-1)     /* an argument is out of range or inconsistent            */
#define HE_FK_EDEVICE (-2)    /* a HIP call failed (no device, launch error, ...)         */
#define HE_FK_ENONFINITE (-3) /* a sample row counts walkers with non-finite ln w / E_L   */
#define HE_FK_EALLDEAD (-4)   /* a sample row has no live walker (all absorbed)          */
#define HE_FK_ESCRATCH (-5)   /* workspace / scratch smaller than the size query returns */

/* ---- trial functions psi_T (theta = {t0, t1, t2, t3, t4, t5}; t5 unused) ---- */
/* exp(-t0 (r1 + r2)).  With Z = 2, ee = 0, t0 = 2 it is exact (E_L = -4);
   with Z = 1, ee = 0, t0 = 1 it is two hydrogen atoms (E_L = -1). */
#define HE_FK_TRIAL_EXPO 0
/* exp(-t0 (r1 + r2)) exp(t2 r12 / (1 + t1 r12))  (Pade-Jastrow, ground state) */
#define HE_FK_TRIAL_PADE 1
/* [exp(-t0 r1 - t3 r2) - exp(-t0 r2 - t3 r1)] exp(t2 r12 / (1 + t1 r12));
   node r1 = r2, the exact node of the 2^3S state (trial functions 3-6 of the
   paper share it) */
#define HE_FK_TRIAL_TRIPLET 2
/* [z2 exp(-t0 r1 - t3 r2) + sym z1 exp(-t0 r2 - t3 r1)] exp(t2 r12 / (1 + t1 r12));
   odd under z -> -z for both electrons (a P_z state, cf. trial function 7) */
#define HE_FK_TRIAL_PZ 3
/* [(t4 - r1) exp(-t0 r1 - t3 r2) - (t4 - r2) exp(-t0 r2 - t3 r1)] exp(t2 r12 / (1 + t1 r12)):
   the paper's trial functions 3-5 for the 2^3S state (r0 = t4, alpha1 = t0, alpha2 = t3;
   no Jastrow factor when t2 = 0); node r1 = r2 */
#define HE_FK_TRIAL_TRIPLET_R0 4
/* (z1 + z2) [exp(-t0 r1 - t3 r2) + exp(-t0 r2 - t3 r1)] exp(t2 r12 / (1 + t1 r12)): the
   paper's trial function 7 for the P_z state ((r1 cos th1 + r2 cos th2) times the symmetric
   exponential pair, alpha1 = t0, alpha2 = t3, no Jastrow factor when t2 = 0); its node is the
   plane z1 + z2 = 0 of the necessary nodal condition z1 = -z2 */
#define HE_FK_TRIAL_PZ_SUM 5

#define HE_FK_FP64 0  /* coordinates, drift, E_L, ln w all binary64                       */
#define HE_FK_MIXED 1 /* coordinates, drift, E_L binary32; ln w, reductions binary64     */

#define HE_FK_NOISE_GAUSS 0 /* Euler-Maruyama: sqrt(dt) xi, xi ~ N(0, I_6) by Box-Muller   */
#define HE_FK_NOISE_PM1 1   /* the paper's walk: sqrt(dt) eps, eps_j = +-1 w.p. 1/2 each   */

#define HE_FK_QUAD_TRAPEZOID 0 /* ln w -= dt/2 [(E_L(Y_k) - e_ref) + (E_L(Y_k+1) - e_ref)]  */
#define HE_FK_QUAD_RIGHT 1     /* ln w -= dt (E_L(Y_k+1) - e_ref): the paper's Riemann sum    */

/* Propagation variants (he_fk_params.flags).
 *
 * HE_FK_FLAG_PLAIN: the plain Feynman-Kac walk of eqs. (2)-(3) with f = 1, the
 *   non-recurrent process that the generalized walk replaces (section "Path
 *   Integral Theory", first paragraphs): Y' = Y + sqrt(dt) xi (no drift) and the
 *   integrand V - e_ref in place of E_L - e_ref.  The start ensemble (|psi_T|^2)
 *   and the node test (absorbing at the node of psi_T) are those of the
 *   generalized walk; el still reports E_L.  Requires drift_limit = 0.
 *
 * HE_FK_FLAG_BRIDGE: node trials only.  Each step that keeps the sign of psi_T
 *   also multiplies the weight by the chance that the path between its end
 *   points did not touch the node, 1 - exp(-2 d d' / dt) (Brownian bridge at a
 *   flat boundary, reflection principle), with the node distance estimated as
 *   d = 1 / |grad ln|Phi|| from the orbital part Phi of the trial function:
 *   ln w += log(-expm1(-2 / (dt |grad ln Phi(Y)| |grad ln Phi(Y')|))), in
 *   binary64.  Exact for the driftless walk at a flat node; an estimate
 *   between the end points of the generalized walk. */
#define HE_FK_FLAG_PLAIN 1
#define HE_FK_FLAG_BRIDGE 2

/*
 * Random stream contract (Philox4x32-10, Salmon et al. SC'11).  The counter of
 * block b is (b, phase, lo32(g), hi32(g)) for global walker id
 * g = walker_offset + i, the key is (lo32(seed), hi32(seed)).  Phase 0: start
 * draw; 1: Metropolis; 2: Gaussian propagation; 3: +-1 propagation.  The
 * propagation draw of global step k depends on k only, so calls are
 * resumable.
 *   contract 1: Gaussian vector k uses blocks 2k, 2k+1; uniforms (w + 1/2) 2^-32
 *               from words (a0,a1), (a2,a3), (b0,b1) (binary32 runs use the top
 *               23 bits: ((w >> 9) + 1/2) 2^-23).
 *   contract 2: Gaussian vector k uses block k; six 21-bit fields
 *               f_j = w_j & (2^21 - 1) (j < 4), f_4 = (w0 >> 21) | ((w1 >> 21) & 1023) << 11,
 *               f_5 = (w2 >> 21) | ((w3 >> 21) & 1023) << 11; uniforms (f + 1/2) 2^-21,
 *               identical in both precisions.
 *   +-1 walk:   step k reads block k / 20, word (k mod 20) / 5, bits 6 (k mod 5) + j.
 * The start ensemble is drawn in binary64 for both precisions (see he_fk_init),
 * so a MIXED and an FP64 run of the same seed start from the same walkers.
 */

typedef struct {
    int32_t trial;        /* HE_FK_TRIAL_* */
    int32_t sym;          /* +1 or -1 (HE_FK_TRIAL_PZ only) */
    int32_t ee;           /* 1: V holds +1/r12; 0: independent electrons */
    int32_t noise;        /* HE_FK_NOISE_* */
    int32_t quad;         /* HE_FK_QUAD_* */
    int32_t contract;     /* 1 or 2 (Gaussian noise only) */
    int32_t precision;    /* HE_FK_FP64 or HE_FK_MIXED */
    int32_t n_metropolis; /* Metropolis steps of the start ensemble (>= 0) */
    int32_t flags;        /* 0 or an OR of HE_FK_FLAG_* (propagation variants) */
    int32_t reserved;     /* must be 0 */
    double Z;             /* nuclear charge (> 0) */
    double theta[6];      /* trial parameters, see HE_FK_TRIAL_* */
    double dt;            /* time step (> 0) */
    double e_ref;         /* trial energy lambda0 of eq. (4); shifts ln w, cancels in E */
    double metropolis_sigma; /* Metropolis proposal width (> 0) */
    double init_sigma;    /* width of the Gaussian the Metropolis chain starts from (> 0) */
    /* drift_limit = a >= 0.  a = 0: the plain discretisation.  a > 0: near the
       singular points of b and E_L (the node of an inexact trial function)
       the drift and the integrand are limited by f = 2 / (1 + sqrt(1 + 2 a dt |b|^2))
       (Umrigar, Nightingale, Runge, J. Chem. Phys. 99, 2865 (1993)):
       Y' = Y + dt f b + sqrt(dt) xi and E_L - e_ref -> f (E_L - e_ref).  f -> 1
       as dt -> 0, so the limit dt -> 0 is unchanged; it keeps a walker that lands
       next to the node from taking an unbounded weight in one step. */
    double drift_limit;
    uint64_t seed;        /* Philox key */
    uint64_t walker_offset; /* global id of walker 0 of this call (shards of one ensemble) */
    int64_t n_walkers;    /* N >= 1 */
} he_fk_params;

/* Walker state, structure of arrays in device memory:
 *   x   [6][N]: x1 y1 z1 x2 y2 z2 rows, binary64 (FP64) or binary32 (MIXED);
 *   lnw [N]   : ln w, binary64.  -inf: absorbed at the node.  NaN: the walker
 *               met a non-finite local energy (kept NaN from then on);
 *   el  [N]   : E_L at the current position, binary64 or binary32 (output). */
typedef struct {
    void* x;
    double* lnw;
    void* el;
} he_fk_walkers;

/*
 * he_fk_init: the start ensemble Y0 ~ psi_T^2 (the start point of eq. (4) is
 * left open by the paper; a |psi_T|^2 start makes L(0) = 0 and E_mixed(0)
 * the variational energy).  Per walker, in binary64 for both precisions:
 * Y = init_sigma * xi(phase 0, Gaussian vector 0, contract 1); then
 * n_metropolis steps with a uniform box proposal of standard deviation
 * metropolis_sigma: Philox block m of phase 1 gives six 16-bit fields f_j
 * (low/high halves of words 0, 1, 2), Y'_j = Y_j + sqrt(3) metropolis_sigma
 * (2 (f_j + 1/2) 2^-16 - 1), accepted iff ln u < 2 (ln|psi(Y')| - ln|psi(Y)|)
 * with u = (w3 + 1/2) 2^-32.  Writes x (rounded to binary32 for MIXED),
 * el = E_L(Y0), lnw = 0.
 * Errors: EINVAL (bad params / NULL pointers), EDEVICE.
 */
int he_fk_init(const he_fk_params* p, const he_fk_walkers* w, void* stream);

/* Bytes of device workspace he_fk_propagate needs (per-block partial sample
   rows); 0 when the arguments are invalid or no device is present. */
size_t he_fk_propagate_workspace_bytes(const he_fk_params* p, int64_t n_steps, int32_t sample_every);

/*
 * he_fk_propagate: advance every walker over global steps [step0, step0 + n_steps)
 * (drifted diffusion after eq. (4), discretised as in the paper's random-walk
 * construction; absorption at the node for the TRIPLET, TRIPLET_R0, PZ and PZ_SUM trials):
 *   Y' = Y + dt b(Y) + sqrt(dt) xi_k,  b = grad ln|psi_T|;
 *   Y = Y' and ln w updated by the quadrature rule, unless sign psi_T(Y') != sign psi_T(Y)
 *   or psi_T(Y') = 0: then the walker is absorbed (lnw = -inf) and stays at Y' (x and el
 *   of an absorbed walker are those of the first position found across the node).
 * With HE_FK_FLAG_PLAIN, b = 0 and the integrand is V - e_ref; with HE_FK_FLAG_BRIDGE
 * the node-touch survival term is added to ln w after the quadrature.
 * samples [n_steps / sample_every + 1][8] (device, binary64): row s is the
 * space average at step step0 + s * sample_every (row 0 = the state on entry):
 *   (m, S0, S1, S2, n_alive, n_nonfinite, n_total, 0) with m = max ln w over
 *   live walkers, S0 = sum e^(lnw - m), S1 = sum e^(lnw - m) E_L,
 *   S2 = sum e^(2 (lnw - m)); so L = m + ln S0 - ln n_total.
 * The reduction tree is fixed, so repeated calls are bitwise identical.
 * ckpt (device, binary64, may be NULL; FP64 precision only):
 *   [n_steps / ckpt_every + 1][7][N], rows x1..z2, lnw at steps step0 + c * ckpt_every.
 * workspace: at least he_fk_propagate_workspace_bytes(p, n_steps, sample_every) bytes.
 *   On return its first bytes hold the per-block partial rows [G][n_samples][8]
 *   (G = that size / (64 n_samples)), each over a fixed subset of walkers, whose
 *   merge is `samples` (usable for block error bars).
 * Constraints: n_steps >= 0, sample_every >= 1, n_steps % sample_every == 0,
 * ckpt_every >= 1 and n_steps % ckpt_every == 0 when ckpt != NULL, step0 >= 0,
 * step0 + n_steps < 2^31.
 * Errors: EINVAL, ESCRATCH, EDEVICE.
 */
int he_fk_propagate(const he_fk_params* p, const he_fk_walkers* w, int64_t step0, int64_t n_steps,
                    int32_t sample_every, double* samples, double* ckpt, int32_t ckpt_every,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * he_fk_propagate_noalloc: he_fk_propagate for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as he_fk_propagate, bitwise,
 * without the workspace: the per-block partial rows live in a static device array
 * of HE_FK_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held from the first call on that
 * GPU until the process ends.  The call allocates nothing (no hipMalloc / hipFree).
 *   - The rows need he_fk_propagate_workspace_bytes(p, n_steps, sample_every) bytes
 *     (64 bytes per block and sample row; a grid has at most one block per resident
 *     slot, so 128 sample rows fit 2048 blocks); a call needing more than
 *     HE_FK_NOALLOC_SCRATCH_BYTES returns HE_FK_ESCRATCH before launching anything.
 *   - The array keeps the last call's partial rows.  Calls that overlap on one GPU
 *     (two streams, two threads) share it and race: serialise them.
 * Errors: as he_fk_propagate (EINVAL, ESCRATCH, EDEVICE).
 */
#define HE_FK_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int he_fk_propagate_noalloc(const he_fk_params* p, const he_fk_walkers* w, int64_t step0, int64_t n_steps,
                            int32_t sample_every, double* samples, double* ckpt, int32_t ckpt_every,
                            void* stream);

/* ---- energy estimators (host only, pure) ---- */
#define HE_FK_E_FD 0     /* E_out[n_samples-1]: e_ref - (L_j - L_{j-1}) / dt_sample            */
#define HE_FK_E_WINDOW 1 /* E_out[1]: e_ref - least-squares slope of L(t) over t in [T/2, T]   */
#define HE_FK_E_FIT 2    /* E_out[2]: {e_ref - b, a} of the least-squares fit L/t = b + a/t,
                            t > 0, weights fit_w[n_samples] (NULL: equal); the paper's
                            "ls fit" with lambda1 = lambda0 - b (Tables 1-5)                 */
#define HE_FK_E_MIXED 3  /* E_out[n_samples]: S1 / S0, the weighted mean local energy       */

/*
 * he_fk_energy: estimators from sample rows (HOST memory, as written by
 * he_fk_propagate and copied back).  Row j is at time t_j = j * dt_sample.
 * aux_out (host, may be NULL): [n_samples][3] = (L_j, S0_j^2 / S2_j, L2_j): the log
 * space average L = m + ln S0 - ln N (eq. (4)'s ln Z(t)), the effective sample size,
 * and the log mean square weight L2 = 2 m + ln S2 - ln N (L2 - 2 L = -ln(ESS / N),
 * the log relative variance of the weights).
 * Errors: EINVAL, ENONFINITE (a row counts non-finite walkers),
 * EALLDEAD (a row has no live walker).  aux_out is filled before these two
 * are reported.
 */
int he_fk_energy(const double* samples, int64_t n_samples, double dt_sample, double e_ref, int32_t method,
                 const double* fit_w, double* E_out, double* aux_out);

/*
 * he_fk_energy_blocks: an estimator and its delete-one-group jackknife standard error
 * from one run.  partials (HOST memory): the per-block partial rows [n_parts][n_samples][8]
 * that he_fk_propagate leaves in its workspace (each block's rows cover a fixed, disjoint
 * set of walkers; n_parts = workspace bytes / (64 n_samples)).  The blocks form
 * G = min(n_groups, n_parts) contiguous groups whose sizes differ by at most one (the
 * larger first); rows merge by rescaling to the larger maximum, as on the device.  The
 * statistic: WINDOW the window energy, FIT lambda1 = e_ref - b, FD the energy of the last
 * sampling interval, MIXED the mixed estimate at the last row (fit_w as for he_fk_energy).
 * est_out (host) [2]: the statistic of all blocks merged, and
 * sqrt((G - 1)/G sum_g (x_g - mean x)^2) over the G replicas x_g without group g.
 * Constraints: n_parts >= 2, n_groups >= 2.
 * Errors: as he_fk_energy on the merged rows or a replica; EINVAL.
 */
int he_fk_energy_blocks(const double* partials, int64_t n_parts, int64_t n_samples, int32_t n_groups,
                        double dt_sample, double e_ref, int32_t method, const double* fit_w, double* est_out);

/* ---- pathwise gradient (adjoint) ---- */
#define HE_FK_GRAD_SCORE 1 /* add the derivative of the |psi_T|^2 start law (score term) */
#define HE_FK_GRAD_MOMENT2 2 /* gL holds 2 n_samples weights: on L_s, then on L2_s = ln <w^2>_s */

/* Bytes of device scratch he_fk_grad needs; 0 on invalid arguments. */
size_t he_fk_grad_scratch_bytes(const he_fk_params* p, int64_t n_steps, int32_t sample_every,
                                int32_t ckpt_every);

/*
 * he_fk_grad: d/d(theta0, theta1) = d/d(alpha, beta) of J = sum_s gL[s] L_s
 * (+ sum_s gL[n_samples + s] L2_s with HE_FK_GRAD_MOMENT2, L2_s = 2 m + ln S2 - ln N,
 * the log of the mean square weight: L2 - 2 L is the log relative variance of the
 * weights, -ln(ESS / N), the objective for tuning psi_T to cut the estimator's variance),
 * L_s the log space average of sample row s of one he_fk_propagate call from
 * step 0 with checkpoints, for the nodeless trials (EXPO, PADE), FP64, no
 * drift limiting.  The derivative is pathwise: start positions (checkpoint
 * row 0) and noise are held fixed, so it is the exact derivative of the
 * discrete map the propagate call computed.  Reverse sweep over the checkpoint
 * segments; each segment is recomputed from its checkpoint into the scratch
 * tape with the noise regenerated from Philox, then one reverse-mode pass
 * through the trial evaluation per step gives grad_Y and d_theta of
 * dt lambda . b + A_j (E_L - e_ref) (lambda the adjoint of the position,
 * A_j the weight of step j's local energy in J).  With ckpt_every = 1 the
 * checkpoints are the whole trajectory (56 bytes per walker-step: 14.7 GB for
 * 2^18 walkers x 1000 steps) and the sweep reads the positions directly, with
 * no recomputation and no tape in the scratch; the result is bitwise that of
 * any other ckpt_every, as the recomputed positions are the stored ones.
 *   ckpt    : device, the checkpoints [n_steps/ckpt_every + 1][7][N] of that call;
 *   samples : device, its sample rows (m and S0 give each walker's share of L_s);
 *   gL      : HOST, [n_steps / sample_every + 1], or twice that with HE_FK_GRAD_MOMENT2;
 *   flags   : an OR of HE_FK_GRAD_SCORE (adds sum_s gL[s] sum_i (p_is - 1/N) 2 d ln|psi(Y0_i)|/d theta,
 *             the derivative through the |psi|^2 law of the start positions; for L2_s the shares
 *             are q_is = w_is^2 / sum_i w_is^2) and HE_FK_GRAD_MOMENT2;
 *   scratch : device, at least he_fk_grad_scratch_bytes(...) bytes;
 *   dtheta  : device, [2] binary64 output (written by the last kernel of the call).
 * Constraints: n_steps % sample_every == 0, n_steps % ckpt_every == 0, and one of
 * ckpt_every, sample_every divides the other; p, seed, walker_offset and n_walkers
 * as in the propagate call.
 * Errors: EINVAL (also node trials, MIXED precision, drift_limit != 0), ESCRATCH, EDEVICE.
 */
int he_fk_grad(const he_fk_params* p, const double* ckpt, const double* samples, const double* gL,
               int64_t n_steps, int32_t sample_every, int32_t ckpt_every, int32_t flags, void* scratch,
               size_t scratch_bytes, double* dtheta, void* stream);

/* Static description of an error code. */
const char* he_fk_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* HE_FK_H */
