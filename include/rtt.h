/*
 * rtt.h - C ABI of the replica-tensor-train (RTT) Monte Carlo library for
 * AMD Instinct MI355X (gfx950).
 *
 * An RTT (Srdinsek, Gouraud, Waintal, "Replica Tensor Train", Sec. 2.2.1) is
 * a tensor train of L cores whose position k reads physical spin pi[k]; the
 * amplitude of a spin configuration s is the product
 *     psi(s) = A_0[s_pi(0)] A_1[s_pi(1)] ... A_{L-1}[s_pi(L-1)]
 * of bond[k] x bond[k+1] matrices, with open boundary bonds
 * bond[0] = bond[L] = 1 (Sec. 2.1).  A spin may be read at several positions
 * (its replica set R_j = pi^{-1}(j)); flipping spin j switches the slice at
 * every position of R_j (the X commutation rule of Sec. 2.2.3).
 *
 * Conventions for every call below
 *   - Status codes: RTT_OK on success, a negative rtt_status otherwise;
 *     rtt_last_error() returns a thread-local message for the last failure.
 *     Argument errors are detected on the host before anything is launched.
 *   - Host pointers are read during the call only; the library keeps its own
 *     copies.  Device pointers are caller-owned and never freed here.
 *   - Spin configurations live in device memory as uint64 words
 *     [W][ceil(N/64)], bit (j % 64) of word (j / 64) holding s_j in {0, 1};
 *     Z_j |s> = (1 - 2 s_j) |s>.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Evaluation and
 *     sampling calls only enqueue work on it and never synchronise; create,
 *     lincomb and destroy synchronise the device.  Workspace a call needs
 *     beyond what a handle already holds (flip-ratio rows for more walkers
 *     than any earlier call, proposal buffers) comes from HIP's
 *     stream-ordered allocator on `stream`, which does not synchronise
 *     either; a handle's workspace is used by one stream at a time, so calls
 *     on one handle (RTT or network) must not overlap on different streams.
 *   - A walker whose amplitude is zero or not finite gets status
 *     RTT_E_NONFINITE in the optional per-walker status array and NaN
 *     outputs; it is never skipped silently and never advanced by sampling.
 */
#ifndef RTT_H
#define RTT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtt_s* rtt_t;       /* packed device cores, schedules, workspace */
typedef struct rtt_ham_s* rtt_ham_t; /* transverse-field Ising Hamiltonian */

typedef enum {
  RTT_F32 = 1,      /* cores rounded to FP32; FP32 matrix cores, FP32 accumulation */
  RTT_BF16 = 2,     /* cores rounded (via FP32) to BF16; activations carried as a
                       hi+lo BF16 pair; FP32 accumulation */
  RTT_FP8_E4M3 = 3  /* cores as OCP e4m3 codes times one power-of-two scale per
                       train position; exact BF16 dequantisation, then as BF16 */
} rtt_dtype;

typedef enum {
  RTT_OK = 0,
  RTT_E_ARG = -1,          /* invalid argument */
  RTT_E_OOM = -2,          /* device allocation failed */
  RTT_E_HIP = -3,          /* a HIP runtime call failed */
  RTT_E_UNSUPPORTED = -4,  /* valid input outside what the library supports */
  RTT_E_NONFINITE = -5     /* per-walker status: zero or non-finite amplitude */
} rtt_status;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* rtt_last_error(void);

/* ABI version; bumped on any incompatible change. */
int32_t rtt_abi_version(void);

/*
 * Build an RTT on the current HIP device (Sec. 2.2.1 definition above).
 *   n_spins  N >= 1 (N <= 1024)
 *   n_cores  L >= 1
 *   pi       host int32[L], values in [0, N); spins read by no position are
 *            allowed (their flip ratio is exactly 1)
 *   bond     host int32[L+1], bond[0] = bond[L] = 1, 1 <= bond[k] <= 256
 *            (<= 128 for RTT_F32)
 *   cores    host double, core k after core k-1, each stored row-major as
 *            [2][bond[k]][bond[k+1]] (slice s = value of the spin read there)
 *   dtype    rtt_dtype
 * The library quantises the cores, packs them into matrix-core operand
 * layouts padded to a power-of-two bond, and builds its contraction schedule.
 * When every bond is at most 4 (the paper's chi = 2 states), evaluation and
 * sampling take vector-ALU kernels on C x C slices instead (C = 2 or 4, FP32
 * arithmetic on the same quantised values); the environment variable
 * RTT_NARROW=0 at creation keeps such a train on the matrix-core kernels.
 * Matrix-core sweeps at padded bonds up to 64 keep the right environments of
 * a few bonds (column checkpoints) on chip between proposals;
 * RTT_CHAIN_CHECKPOINTS=0 at creation
 * makes every proposal contract its columns from the right boundary (the
 * batched entry points always do, so results then match them bit for bit).
 * The batched entry points always use the matrix-core kernels.
 * RTT_E_UNSUPPORTED if the working set of one walker exceeds on-chip memory.
 */
rtt_status rtt_create(int32_t n_spins, int32_t n_cores, const int32_t* pi,
                      const int32_t* bond, const double* cores, int32_t dtype,
                      rtt_t* out);

/*
 * Linear combination psi = sum_a coeffs[a] psi^a (Sec. 3.2, lin_comb
 * equation) of n_terms RTTs that share N, L, pi, the padded bond and dtype.
 * The new handle owns copies; the terms may be destroyed afterwards.
 * coeffs: host double[n_terms].  RTT_E_ARG on mismatched terms.
 */
rtt_status rtt_lincomb(int32_t n_terms, const rtt_t* terms, const double* coeffs,
                       rtt_t* out);

rtt_status rtt_destroy(rtt_t h);

/* info (host int32[10]): N, L, padded bond, dtype, n_terms, words per walker,
   cut bond of the flip-ratio schedule, rows per walker and row group, row
   groups, and the width C of the narrow-bond path (0 when the matrix-core
   kernels run; see rtt_create). */
rtt_status rtt_info(rtt_t h, int32_t* info);

/*
 * Quantised core values of term `term` exactly as the device uses them
 * (FP8 scale applied), written to host `out` in the rtt_create layout.  The
 * values are read back from device memory and unpacked from the fragment
 * layout, so this also checks the packing.  Synchronises.
 */
rtt_status rtt_get_cores(rtt_t h, int32_t term, double* out);

/*
 * H = J sum_<ij> Z_i Z_j - h sum_i X_i on an Lx x Ly square lattice, sites in
 * raster order i = y*Lx + x (Sec. 4, Ising model equation).  With periodic != 0
 * wrap-around bonds are added along each side of length >= 3.
 */
rtt_status rtt_tfim_create(int32_t Lx, int32_t Ly, int32_t periodic, double J,
                           double h, rtt_ham_t* out);
rtt_status rtt_tfim_destroy(rtt_ham_t ham);

/*
 * Evaluate W walkers at the configurations `spins` (device, read only).
 * Every output is an optional device pointer (NULL = not wanted):
 *   logabs  double[W]      log|psi(s)|
 *   sign    int8[W]        sign of psi(s) (+1 / -1)
 *   logratio double[W][N]  log|r_j|, r_j = psi(s with s_j flipped) / psi(s)
 *                          (flip at every replica of j, Sec. 2.2.3)
 *   rsign   int8[W][N]     sign of r_j
 *   eloc    double[W]      local energy sum_s' H_{s s'} psi(s') / psi(s)
 *                          = J sum z_i z_j - h sum_j r_j (needs ham)
 *   status  int32[W]       RTT_OK or RTT_E_NONFINITE per walker
 * ham may be NULL unless eloc is requested.
 */
rtt_status rtt_evaluate(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins,
                        double* logabs, int8_t* sign, double* logratio, int8_t* rsign,
                        double* eloc, int32_t* status, void* stream);

/*
 * rtt_evaluate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, outputs and errors as rtt_evaluate, the same kernels and
 * bit-identical results, but the flip-ratio workspace is a fixed 64 MiB
 * device array inside the library (one per GPU, held until the process
 * ends) instead of the handle's own, and no call allocates or frees
 * anything.  The workspace needed is 2 * T * groups * W * slots * (4 * bond
 * + 4) bytes (T terms, padded bond, and groups and slots per walker as
 * rtt_info reports them); a larger W gives RTT_E_ARG with the largest W
 * this state allows per call (e.g. about 1600 walkers of the 8x8, bond-64
 * train, 25 of the 16x16 bond-256 four-term combination), checked before
 * any launch.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams, threads or handles) race and must
 * be ordered by the caller.  Nothing in the array needs to start at zero.
 * Trains on the narrow-bond path need no workspace.
 */
rtt_status rtt_evaluate_noalloc(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins,
                                double* logabs, int8_t* sign, double* logratio, int8_t* rsign,
                                double* eloc, int32_t* status, void* stream);

/* Amplitudes only: log|psi| and sign for W walkers (device pointers). */
rtt_status rtt_amplitudes(rtt_t h, int32_t W, const uint64_t* spins, double* logabs,
                          int8_t* sign, void* stream);

/* All N single-flip ratios per walker (device pointers, [W][N]). */
rtt_status rtt_flip_ratios(rtt_t h, int32_t W, const uint64_t* spins,
                           double* logratio, int8_t* rsign, void* stream);

/* Local energies (device double[W]). */
rtt_status rtt_local_energy(rtt_t h, rtt_ham_t ham, int32_t W, const uint64_t* spins,
                            double* eloc, void* stream);

/*
 * n_sweeps single-spin-flip Metropolis sweeps on P(s) = |psi(s)|^2 / Z
 * (Sec. 3.3).  One sweep proposes each spin once, in order of its first
 * train position (spins read by no position last); the move is accepted iff
 * u < r_j^2, with u = (x >> 11) * 2^-53 and x word 0 of Philox4x64-10 under
 * key (seed, rng_stream) and counter (walker index, sweep0 + t, j, 0).
 * Each proposal's flipped amplitude is contracted from the prefix of the
 * spin's first position to a right environment of the current configuration
 * (the right boundary, or a checkpoint bond past the spin's last position
 * kept on chip since an earlier proposal), so the rounding of an amplitude
 * depends on which checkpoints are valid: decisions agree with an exact
 * evaluation except at near-ties (|u - r^2| within the FP32/BF16 error).
 *   spins    device uint64[W][ceil(N/64)], updated in place
 *   logabs   device double[W] or NULL: log|psi| of the final configuration
 *   sign     device int8[W] or NULL
 *   accepts  device uint32[W] or NULL: accepted moves, added to the input
 *   status   device int32[W] or NULL
 */
rtt_status rtt_mcmc_sweep(rtt_t h, int32_t W, uint64_t* spins, double* logabs,
                          int8_t* sign, uint64_t seed, uint64_t rng_stream,
                          uint64_t sweep0, int32_t n_sweeps, uint32_t* accepts,
                          int32_t* status, void* stream);

/*
 * Dual Monte Carlo estimators (Sec. 3.3, "Dual Monte Carlo"): walkers s
 * sampled from P^a = |psi^a|^2 / Z_a (e.g. by rtt_mcmc_sweep on psi^a),
 * evaluated against each of M target states psi^b_m:
 *   ratio[m][w] = psi^b_m(s_w) / psi^a(s_w)
 *   mixed[m][w] = sum_t H_{s_w,t} psi^b_m(t) / psi^a(s_w)   (mixed local energy)
 * Their averages over P^a are the row a of the un-symmetrised overlap and
 * Hamiltonian matrices S~_ab, H~_ab of the physical-space optimisation
 * (reduce each row with rtt_energy_reduce).  A target may be psi^a itself
 * (ratio 1, mixed = E_loc) or any RTT / linear combination with the same
 * spin count.
 *   targets    host array of M handles, M >= 1
 *   ham        TFIM on a lattice of N sites
 *   spins      device uint64[W][ceil(N/64)]
 *   logabs_a, sign_a  device double[W], int8[W]: log|psi^a| and sign of the
 *              walkers (as rtt_mcmc_sweep or rtt_amplitudes leave them)
 *   ratio, mixed  device double[M][W] (row m for target m)
 *   status     device int32[W] or NULL: 0, or RTT_E_NONFINITE (-5) if the
 *              sampled or any target amplitude is zero or non-finite (that
 *              walker's outputs are NaN)
 * Each target keeps a W-sized workspace, grown on demand in stream order;
 * calls on one target must not overlap.  Errors: RTT_E_ARG for null
 * pointers, M < 1, W < 1, invalid handles or spin counts differing from the
 * lattice; otherwise as rtt_evaluate.
 */
rtt_status rtt_mixed_estimators(int32_t M, const rtt_t* targets, rtt_ham_t ham, int32_t W,
                                const uint64_t* spins, const double* logabs_a,
                                const int8_t* sign_a, double* ratio, double* mixed,
                                int32_t* status, void* stream);

/*
 * Tensor-train rounding on the host (FP64): right-to-left orthogonalisation
 * by Householder QR, then left-to-right truncated SVDs keeping at most
 * chi_max singular values per bond and none below rel_tol times the
 * largest.  Compression step of the replica-space optimisation (Sec. 3.1).
 *   bond, cores   host, rtt_create layout (bond[0] = bond[L] = 1)
 *   bond_out      host int32[L+1]; cores_out host double[cap]
 *   n_out         doubles written (or needed, with RTT_E_ARG when cap is short)
 * Synchronous, no GPU work.  Errors: RTT_E_ARG for bad bonds, non-finite
 * entries, chi_max < 1, rel_tol < 0 or too small an output.
 */
rtt_status rtt_tt_round(int32_t n_cores, const int32_t* bond, const double* cores,
                        int32_t chi_max, double rel_tol, int32_t* bond_out,
                        double* cores_out, int64_t cap, int64_t* n_out);

/*
 * One replica-space power step for the TFIM (Sec. 3.1, optimisation in the
 * replica space, with the Sec. 2.2.3 commutation rules): for the train phi
 * of path pi, returns round(phi - tau * H-bar phi) where
 *   H-bar = J sum_<ij> Zbar_i Zbar_j - h sum_j Xbar_j,
 * Xbar_j swaps the slices of every core reading spin j, Zbar_i changes the
 * sign of slice 1 of the first core reading spin i, so that C phi' =
 * (1 - tau H) C phi before compression.  The terms of H-bar phi are summed
 * two by two with a rounding (chi_max, rel_tol) after each sum; the final
 * difference is rounded once more.  Lattice Lx x Ly (= n_spins sites) with
 * the bonds of rtt_tfim_create; every spin must be read by some position.
 * Host FP64, synchronous; outputs and errors as rtt_tt_round.
 */
rtt_status rtt_tfim_power_step(int32_t n_spins, int32_t n_cores, const int32_t* pi,
                               const int32_t* bond, const double* cores, int32_t Lx,
                               int32_t Ly, int32_t periodic, double J, double h,
                               double tau, int32_t chi_max, double rel_tol,
                               int32_t* bond_out, double* cores_out, int64_t cap,
                               int64_t* n_out);

/*
 * A sum of Pauli strings applied to a train (Sec. 2.2.3 replica-space
 * operators, Sec. 3.1 power method, Sec. 4.1.3 operators routed to one part
 * of the path): returns round(alpha phi + beta sum_t coeffs[t] O_t phi).
 *   ops     host uint8[n_terms][n_cores]: the string O_t per train position,
 *           0 = identity, 1 = X (slices swapped), 2 = Z (slice 1 negated),
 *           3 = X Z (slice 1 negated, then slices swapped)
 *   coeffs  host double[n_terms]
 * The terms are summed two by two in index order with a rounding (chi_sum,
 * rel_tol) after each sum; the result is scaled by beta, alpha phi is added
 * when alpha != 0, and the whole is rounded to (chi_max, rel_tol).  Rounding
 * the partial sums to the final rank discards most of a power step; a
 * chi_sum of a few times chi_max keeps it.  alpha = 1,
 * beta = -tau with the strings of a replica Hamiltonian is one power step
 * phi - tau H-bar phi; alpha = 0, beta = 1 applies an operator.
 * Host FP64, synchronous; outputs as rtt_tt_round.  Errors: RTT_E_ARG for
 * n_terms < 1, chi_sum < 1, an op above 3, non-finite coefficients, alpha
 * or beta, and
 * the train errors of rtt_tt_round.
 */
rtt_status rtt_pauli_apply(int32_t n_cores, const int32_t* bond, const double* cores,
                           int32_t n_terms, const double* coeffs, const uint8_t* ops,
                           double alpha, double beta, int32_t chi_max, int32_t chi_sum,
                           double rel_tol, int32_t* bond_out, double* cores_out, int64_t cap,
                           int64_t* n_out);

/*
 * A linear combination of trains on one path, compressed (the final
 * compression of the physical-space combination sum_a c_a psi^a, Sec. 4.3,
 * and of stochastic Gram-Schmidt, Sec. 3.3): round(sum_m coeffs[m] phi_m).
 *   bonds   host int32[n_trains][n_cores+1], each with bond[0] = bond[L] = 1
 *   cores   host array of n_trains pointers, each to a train in rtt_create layout
 * The trains are summed two by two in index order with a rounding (chi_max,
 * rel_tol) after each sum, then rounded once more.  Host FP64, synchronous;
 * outputs as rtt_tt_round.  Errors: RTT_E_ARG for n_trains < 1, non-finite
 * coefficients and the train errors of rtt_tt_round.
 */
rtt_status rtt_tt_combine(int32_t n_trains, int32_t n_cores, const int32_t* bonds,
                          const double* const* cores, const double* coeffs, int32_t chi_max,
                          double rel_tol, int32_t* bond_out, double* cores_out, int64_t cap,
                          int64_t* n_out);

/*
 * Compensated (Neumaier) FP64 reduction of x[n] (device): out[0] = sum x,
 * out[1] = sum x^2, out[2] = number of finite entries summed (device
 * double[3]).  Non-finite entries are skipped and not counted.
 */
rtt_status rtt_energy_reduce(int32_t n, const double* x, double* out, void* stream);

/*
 * Compensated (Neumaier) FP64 sums of row products (device buffers):
 *   out[2 (a B + b)]     = sum_w x[a][w] * y[b][w]
 *   out[2 (a B + b) + 1] = number of w whose product is finite (summed)
 * for a < A, b < B; x double[A][W], y double[B][W], out double[A][B][2].
 * With y = NULL (and B = 1) the rows of x are summed alone.  Non-finite
 * terms are skipped and not counted.  These are the averages of dual Monte
 * Carlo (Sec. 3.3): rows of S~ and H~ from the estimators of
 * rtt_mixed_estimators, and, for states that differ from the sampled one
 * by diagonal (Z) operators (Sec. 4.1.3), S_ab = <r_a r_b> and
 * H_ab = <r_a m_b> from one chain.  Stream-ordered; RTT_E_ARG for A, B or
 * W < 1, null x or out, or y = NULL with B != 1.
 */
rtt_status rtt_pair_sums(int32_t A, int32_t B, int32_t W, const double* x, const double* y, double* out,
                         void* stream);

/*
 * Batches: many independent RTT Monte Carlo runs of uneven size stepped
 * together in one captured HIP graph of persistent kernels.
 *
 * rtt_batch_create: n >= 1 runs; run b uses RTT rtts[b], Hamiltonian hams[b]
 *   (its lattice must have the RTT's N sites), walkers[b] >= 1 walkers whose
 *   spins live at spins[b] (device uint64[walkers[b]][ceil(N/64)], updated in
 *   place) and whose local energies are written to eloc[b] (device
 *   double[walkers[b]]).  rtts, hams, walkers, spins, eloc are host arrays of
 *   length n; the device buffers are caller-owned and must stay valid, at the
 *   same addresses, for the life of the batch.  Run b draws its Philox
 *   uniforms under key (seed, b).  Handles of the RTTs and Hamiltonians must
 *   outlive the batch.
 * rtt_batch_step: n_sweeps Metropolis sweeps of every walker of every run
 *   (sweep numbers continue from the previous step), then local energies of
 *   every walker, then per-run sums into esum (device double[n][3]: sum of
 *   E_loc, sum of E_loc^2, number of finite values; may be NULL).  The first
 *   call for a given (n_sweeps, esum) captures the graph (this synchronises);
 *   later calls only launch it on `stream`.
 * rtt_batch_autotune: times every launch shape (bond classes one after the
 *   other on the whole GPU, or concurrently on graph branches with compute
 *   units shared in proportion to their work; 1..4 persistent blocks per
 *   compute unit) with `reps` steps each and keeps the fastest; then, class
 *   by class, the sampler's tile: 16 walkers per block, or 32 walkers (two
 *   matrix-core column groups sharing every core fragment a wave loads)
 *   where every member's sampling state fits on chip in the same layout
 *   (padded bonds 32 and 128).  Results do not depend on these choices, bit
 *   for bit.  The choice is appended as one JSON line to cache_path (NULL:
 *   no file): batch signature, shape, per-class walkers per block, number
 *   of trials (each = one capture, one warm-up step and `reps` timed steps),
 *   time per step.  The timed steps advance the chains.  choice (host
 *   int32[2], may be NULL) receives (concurrent, blocks per compute unit).
 *   Synchronises.  The environment variable RTT_BATCH_TILE=32 at
 *   rtt_batch_create starts the eligible classes at 32 walkers per block
 *   (16 otherwise), the tile used until an autotune changes it.
 */
typedef struct rtt_batch_s* rtt_batch_t;

rtt_status rtt_batch_create(int32_t n, const rtt_t* rtts, const rtt_ham_t* hams,
                            const int32_t* walkers, uint64_t* const* spins,
                            double* const* eloc, uint64_t seed, rtt_batch_t* out);
rtt_status rtt_batch_step(rtt_batch_t b, int32_t n_sweeps, double* esum, void* stream);
rtt_status rtt_batch_autotune(rtt_batch_t b, int32_t n_sweeps, int32_t reps,
                              const char* cache_path, int32_t* choice, void* stream);
rtt_status rtt_batch_destroy(rtt_batch_t b);

/*
 * Learned multi-spin proposal (a sampler for P = |psi|^2 / Z, Sec. 3.3; the
 * paper leaves the proposal open).  Network: input z = 1 - 2 s on the
 * periodic Lx x Ly lattice (Lx, Ly >= 3, Lx*Ly <= 256), three 3x3 circular
 * convolutions with 32 channels and SiLU, a 1x1 head with 9 outputs per
 * site: o[0] centre logits, o[1..8] logits of the move size k = 1..8.
 * params (host double[19113]): W1[32][1][3][3], b1[32], W2[32][32][3][3], b2,
 * W3[32][32][3][3], b3, Wh[9][32], bh[9], row-major, concatenated.  The
 * library keeps FP32 master weights and uses them rounded to BF16 (FP32
 * accumulation) in every forward pass; in the proposal and forward kernels
 * the two 32-channel layers run on the BF16 matrix cores with each
 * activation split into three BF16 parts, which keeps FP32 accuracy.
 * A move samples a centre c ~ softmax(o[0]) and k ~ softmax(o[1..8][c]) and
 * flips the first k sites of the spiral (dx,dy) = (0,0),(1,0),(1,1),(0,1),
 * (-1,1),(-1,0),(-1,-1),(0,-1) around c.  It is accepted iff
 *   u < |psi(s')/psi(s)|^2 q(S|s') / q(S|s),
 * q(S|.) being the exact probability of the flipped set S (summed over every
 * (c', k) giving S).  Uniforms: word 0 of Philox4x64-10, key (seed,
 * rng_stream), counter (walker, step, 2^32 + i, 0), i = 0 centre, 1 size,
 * 2 acceptance; inverse-CDF sampling.
 */
typedef struct rtt_net_s* rtt_net_t;

rtt_status rtt_net_create(int32_t Lx, int32_t Ly, const double* params, rtt_net_t* out);
rtt_status rtt_net_destroy(rtt_net_t net);
/* which = 0: FP32 master weights, 1: the BF16-rounded weights in use (host double[19113]) */
rtt_status rtt_net_get_params(rtt_net_t net, int32_t which, double* out);
/* head outputs for W configurations: device float[W][9][Lx*Ly] */
rtt_status rtt_net_forward(rtt_net_t net, int32_t W, const uint64_t* spins, float* out, void* stream);
/*
 * One learned-proposal Metropolis-Hastings step for W walkers.
 *   spins   device uint64[W][ceil(N/64)], updated in place
 *   logabs, sign  device in/out: log|psi| and sign of the current spins
 *           (e.g. from rtt_amplitudes or rtt_mcmc_sweep); updated on acceptance
 *   moves   device int32[W] or NULL: c | (k << 16) proposed
 *   accept_prob device float[W] or NULL: min(1, MH ratio)
 *   before  device uint64[W][ceil(N/64)] or NULL: the states the moves were
 *           proposed at (the training inputs)
 *   accepts device uint32[W] or NULL (incremented), status int32[W] or NULL
 */
rtt_status rtt_mh_learned_step(rtt_t h, rtt_net_t net, int32_t W, uint64_t* spins, double* logabs,
                               int8_t* sign, uint64_t seed, uint64_t rng_stream, uint64_t step,
                               int32_t* moves, float* accept_prob, uint64_t* before,
                               uint32_t* accepts, int32_t* status, void* stream);
/*
 * Gradient (device float[19113]) of sum_b c_b log q(c_b, k_b | s_b) with
 * c_b = -(accept_prob_b * k_b - baseline) / B: the score-function estimate
 * of minus the expected accepted move size.  spins are the states s_b the
 * moves were proposed at.  baseline is the library's running mean of
 * accept_prob * k.
 */
rtt_status rtt_net_grad(rtt_net_t net, int32_t B, const uint64_t* spins, const int32_t* moves,
                        const float* accept_prob, float* grad, void* stream);
/* One training step: the gradient above, then the baseline update
   (0.9 old + 0.1 batch mean) and one Adam step (beta1, beta2, eps) on the
   master weights with learning rate lr. */
rtt_status rtt_net_train(rtt_net_t net, int32_t B, const uint64_t* spins, const int32_t* moves,
                         const float* accept_prob, float lr, float beta1, float beta2, float eps,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RTT_H */
