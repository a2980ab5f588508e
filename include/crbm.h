/*
 * crbm.h -- C ABI of the MI355X (gfx950) hot path of convolutional-RBM-aided
 * Monte Carlo (Alcalde Puente & Eremin, arXiv:2008.05401).
 *
 * The library samples P(x) ~ exp(-beta E(x)) on an L x L periodic lattice
 * with many independent Markov chains.  One "sweep" of a chain is
 *   1. gibbs_k block-Gibbs steps v -> h -> v' of the CRBM (App. B, Gibbs
 *      sampling; conditionals P(h|v), P(v|h) of the convolutional energy
 *      Eq. (energy_CRBM)), which propose x';
 *   2. the CRBM free energy F(x') of Eq. (free-energy_CRBM);
 *   3. the target: the Ising energy E(x') of Sec. III (integer, exact), or the
 *      Kitaev gauge-field weight S(x') = -beta F(x') of Sec. IV from the FP64
 *      singular values of the Majorana hopping block;
 *   4. the Metropolis-Hastings test of Eq. (acceptance) with one replica being
 *      the CRBM: log r = log P(x') - log P(x) + F(x') - F(x); accept iff
 *      log u < log r;
 *   5. observables of the state after the sweep (after burn-in).
 *
 * Conventions common to every entry point
 *   - Pointers marked "device" are HIP device pointers owned by the caller;
 *     the library allocates no device memory.  Pointers marked "host" are
 *     ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All calls are asynchronous with respect to the host and ordered on
 *     that stream, unless stated otherwise.
 *   - Spin states are int8 +-1 with layout [chain][C][L][L], row-major.
 *     The CRBM works on v = (s+1)/2 (App. A).  Ising uses C = 1.  Kitaev uses
 *     C = 3 (bond variables u_x, u_y, u_z of unit cell (i,j), see below) or
 *     C = 1 (only the z-bond field eta, u_x = u_y = +1, as in Sec. IV).
 *   - CRBM filters are float32 W[K][C][Lw][Lw]; the "wrap around convolution"
 *     is a cross-correlation anchored at the filter's top-left element:
 *       a[k][i][j] = hbias[k] + sum_{c,a,b} W[k][c][a][b] v[c][(i+a)%L][(j+b)%L]
 *     and the hidden->visible pass is its exact adjoint:
 *       b[c][x][y] = vbias[c] + sum_{k,a,b} W[k][c][a][b] h[k][(x-a)%L][(y-b)%L].
 *   - Random numbers: Philox4x32-10 with key = seed and counter
 *     (unit>>2, sweep, chain, tag), word unit&3; tag = stream | substep<<8,
 *     streams INIT=0, HID=1, VIS=2, MH=3.  Hidden unit index
 *     (k*L+i)*L+j, visible unit index (c*L+i)*L+j.  A unit is on iff
 *     (x+0.5)/2^32 < sigmoid(pre-activation); the MH uniform is the 53-bit
 *     number from words 0 and 1 of unit group 0.  The initial state takes
 *     s = +1 iff the top bit of its INIT word is set.
 *   - Every entry point validates its arguments on the host and returns a
 *     negative crbm_status on error without launching anything; the message
 *     is available from crbm_last_error().  Faults of launched kernels
 *     surface as CRBM_EHIP at the next call that synchronises.
 *   - Kitaev lattice: unit cell (i,j) holds a black site b and a white site w;
 *     the z bond joins b(i,j)-w(i,j), the x bond b(i,j)-w(i,(j+1)%L), the y
 *     bond b(i,j)-w((i+1)%L,j).  M[b,w] = 2 J_alpha u_alpha (N x N, N = L^2).
 */
#ifndef CRBM_H
#define CRBM_H

#include <stddef.h>
#include <stdint.h>

#ifndef CRBM_API
#define CRBM_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRBM_OK = 0,
    CRBM_EINVAL = -1,      /* invalid argument (shape, size, null pointer, range) */
    CRBM_EBUDGET = -2,     /* workspace too small */
    CRBM_EHIP = -3,        /* a HIP runtime call failed */
    CRBM_EUNSUPPORTED = -4 /* valid but not supported by this library (e.g. LDS too small) */
} crbm_status;

/* CRBM_GIBBS: no target; every proposal is accepted, so the chain is the plain
 * block-Gibbs chain of the CRBM (App. B) -- the sampler of the replay buffer of
 * Alg. 1 and the "uncorrected" RBM of App. B.  C = 1 or 3; the Ising
 * observables of channel 0 are still accumulated. */
typedef enum { CRBM_ISING = 0, CRBM_KITAEV = 1, CRBM_GIBBS = 2 } crbm_target;

/* CRBM parameters theta = (W, hbias, vbias); all device, float32.
 * K in [1, 64], C in {1, 3}, Lw in [1, 8] and Lw <= L.
 * The locally connected CRBM of Sec. IV.B (open boundaries) sets n_edge >= 1:
 * W and hbias then hold 1 + 2 n_edge filter banks; bank 0 is shared by the bulk
 * hidden columns, banks 1..n_edge belong to the hidden columns 0..n_edge-1
 * (left side) and banks n_edge+1..2 n_edge to the columns L-n_edge..L-1 (right
 * side); 0 <= n_edge <= 4 and 2 n_edge <= L.  open_cols = 1 stops the filter
 * windows at the column edge (visible columns past it count as v = 0) instead
 * of wrapping; rows always wrap.  A zero-initialised tail (open_cols = n_edge
 * = 0) is the periodic CRBM of Eq. (energy_CRBM). */
typedef struct {
    int32_t K, C, Lw;
    const float* W;     /* device [banks][K][C][Lw][Lw], banks = 1 + 2 n_edge */
    const float* hbias; /* device [banks][K] */
    const float* vbias; /* device [C] */
    int32_t open_cols;  /* 0: windows wrap in both directions; 1: open columns */
    int32_t n_edge;     /* unshared banks per side */
    int32_t dense;      /* 1: the fully connected RBM (FRBM) of the Sec. IV
                           comparison instead of a convolution: K in [1, 256]
                           hidden units each connected to all C L^2 visible
                           units, Lw = L, W [K][C][L][L], hbias [K], vbias
                           [C][L][L] (one bias per visible unit); open_cols =
                           n_edge = 0 */
} crbm_params;

/* One job: n_chains chains on an L x L lattice.
 * T[g] > 0 is chain g's temperature.  Chain g uses the Philox chain index
 * chain_offset + g, so a chain's trajectory depends only on (seed, its index,
 * sweep number), never on how jobs are batched.
 *
 * rbm_state selects the form of the CRBM move (App. B):
 *   NULL     - the CRBM replica is refreshed from the physical state before
 *              every sweep: gibbs_k Gibbs steps from x give x', accepted with
 *              the probability of Eq. (acceptance);
 *   non-NULL - every chain keeps a persistent CRBM replica y (parallel
 *              tempering with an exchange correction): each sweep advances y
 *              by gibbs_k Gibbs steps to y' and exchanges it with x with the
 *              same probability; accepted: x <- y', y <- x; rejected: y <- y'.
 *              With init_state = 1 crbm_init copies the initial state into
 *              rbm_state; otherwise the caller provides it.  Not allowed
 *              with CRBM_GIBBS. */
typedef struct {
    int32_t target;        /* crbm_target */
    int32_t L;             /* lattice side, 1 <= L <= 256 */
    int32_t n_chains;      /* >= 1 */
    int32_t gibbs_k;       /* Gibbs steps per proposal, >= 1 */
    int32_t burnin_sweeps; /* sweeps with index < burnin are not measured */
    int32_t init_state;    /* 1: crbm_init fills `state` from the INIT stream */
    uint32_t chain_offset; /* Philox chain index of chain 0 */
    int32_t boundary;      /* target lattice: 0 periodic; 1 open columns (Sec. IV.B):
                              the Ising bond / the Kitaev x bond from column L-1
                              to column 0 is absent, rows stay periodic */
    uint64_t seed;         /* Philox key */
    double J[3];           /* Ising: J[0] is J. Kitaev: J_x, J_y, J_z */
    const double* T;       /* device [n_chains] temperatures */
    int8_t* state;         /* device [n_chains][C][L][L], +-1, read and written */
    int8_t* rbm_state;     /* device [n_chains][C][L][L] or NULL; see below */
    void* workspace;       /* device, >= crbm_workspace_size() bytes */
    size_t workspace_bytes;
    double mh_band_min;    /* >= 0: least half-width of the band of |log r - log u|
                              inside which an MH decision is taken again on the
                              exact route (Ising: FP64 free energies of both
                              states; Kitaev: singular values of M by one-sided
                              Jacobi for both states).  0 leaves the band to the
                              rigorous error bounds of the fast route; a huge value
                              sends every decision through the exact route (for
                              tests).  The zero-initialised tail of a desc is 0. */
} crbm_batch_desc;

/* Per-chain record, kept in the workspace; read with crbm_read_stats.
 * Sums cover the measured sweeps (sweep index >= burnin_sweeps) and use the
 * state after each sweep. Ising sums are exact integers in units of J. */
typedef struct {
    int64_t sweeps;       /* sweeps done */
    int64_t n_acc;        /* accepted proposals (all sweeps) */
    int64_t n_meas;       /* measured sweeps */
    int64_t n_recheck;    /* decisions re-evaluated in FP64 (diagnostic) */
    int64_t sumE, sumE2;  /* Ising: sum E/J, sum (E/J)^2 */
    int64_t sumM, sumAbsM, sumM2;
    int64_t E;            /* Ising E/J of the current state */
    double F;             /* CRBM free energy of the current state */
    double S;             /* Kitaev -beta F_gauge of the current state */
    double Ef;            /* Kitaev fermion energy -sum eps/2 tanh(beta eps/2) */
    double Cf;            /* Kitaev sum (beta eps/2)^2 / cosh^2(beta eps/2) */
    double kE, kE2, kCf;  /* Kitaev sums of Ef, Ef^2, Cf */
    double F_bound;       /* bound on |F - F_exact| of the cached F (0: exact FP64) */
    int64_t n_swap;       /* accepted temperature swaps (crbm_tempering_swap) */
    double S_bound;       /* Kitaev: bound on |S - S_exact| of the cached S from
                             the error analysis of the eigen-step; 0 when S
                             comes from the one-sided Jacobi re-check route */
} crbm_chain_stats;

typedef struct crbm_ctx crbm_ctx; /* opaque host-side handle */

/* Bytes of device workspace a job needs (per-chain records plus internal
 * buffers: the bit-packed Ising kernel's filter tables, the Kitaev singular
 * values and eigen-step scratch).  Returns 0 for invalid arguments. Host
 * only, no device work.
 * Kitaev jobs run up to L = 24; the workspace holds an N x N FP64 matrix per
 * chain (N = L^2; 2.7 MB per chain at L = 24, 166 KB at L = 12): M of the
 * Jacobi re-check route, and beyond L = 12 also M^T M of the eigen-step
 * (up to L = 12 that stays in LDS). */
CRBM_API size_t crbm_workspace_size(const crbm_params* params, const crbm_batch_desc* desc);

/* Create a job handle: copies `params`/`desc` (the pointed-to device buffers
 * must stay valid until crbm_destroy), optionally fills the initial state,
 * computes F and the target of every chain's state and zeroes the sums.
 * For jobs on the bit-packed Ising kernel (C = 1, periodic, L a power of two
 * from 8 to 256, Lw <= 6) it also builds, once, the kernel's tables of the
 * filters (subset sums of every filter row, error bands) in the workspace:
 * the filters and biases are therefore read at crbm_init and must not change
 * while the job lives (create a new job for new parameters).
 * Sweep numbering starts at 0. Asynchronous on `stream`. */
CRBM_API crbm_status crbm_init(crbm_ctx** out, const crbm_params* params, const crbm_batch_desc* desc, void* stream);

/* Advance every chain of the job by n_sweeps >= 0 sweeps (steps 1-5 above).
 * Asynchronous on the job's stream; updates `state` and the workspace. */
CRBM_API crbm_status crbm_propose_accept(crbm_ctx* ctx, int32_t n_sweeps);

/* Advance several jobs by n_sweeps each in shared launches (continuous
 * batching). All jobs must use the same stream. */
CRBM_API crbm_status crbm_propose_accept_many(crbm_ctx* const* ctxs, int32_t n_ctx, int32_t n_sweeps);

/* Sweep blocks as a HIP graph: crbm_graph_create captures n_blocks >= 1
 * launches of crbm_propose_accept_many(ctxs, n_ctx, sweeps_per_block) (same
 * rules for the job list) into an executable graph, without running them;
 * crbm_graph_launch enqueues the graph on the jobs' stream and counts
 * n_blocks * sweeps_per_block sweeps for every job.  A launch does exactly
 * what the same eager calls do (states, sums and random streams live in the
 * jobs' device memory, not in the graph), so eager calls, tempering swaps,
 * trace changes and graph launches may be interleaved in stream order.  The
 * jobs must outlive the graph; the graph is bound to the tile shapes chosen
 * when it was captured.  Host memory and one HIP graph per handle;
 * crbm_graph_destroy releases both. */
typedef struct crbm_graph crbm_graph;
CRBM_API crbm_status crbm_graph_create(crbm_graph** out, crbm_ctx* const* ctxs, int32_t n_ctx, int32_t n_blocks,
                                       int32_t sweeps_per_block);
CRBM_API crbm_status crbm_graph_launch(crbm_graph* graph);
CRBM_API crbm_status crbm_graph_destroy(crbm_graph* graph);

/* One round of temperature swaps of parallel tempering (App. B, Eq.
 * (acceptance) between two physical temperatures), stream-ordered after the
 * job's sweeps.  The job's chains form a grid chain = rung * n_ladders +
 * ladder (n_chains must be a multiple of n_ladders); round r pairs the rungs
 * (q, q+1) for q = r % 2, r % 2 + 2, ... of every ladder.  For a pair (a, b):
 *   Ising:  log A = J (1/T_a - 1/T_b) (E_a - E_b)
 *   Kitaev: log A = S_a(x_b) + S_b(x_a) - S_a(x_a) - S_b(x_b), with
 *           S_T(x) = sum_lambda log 2cosh(eps_lambda(x) / (2T)) from the
 *           singular values kept in the workspace;
 * the pair swaps its physical states iff log u < log A, u the 53-bit uniform
 * of Philox counter (0, r, chain_offset + a, 4).  The cached E, F, F_bound
 * (and singular values; S, Ef, Cf recomputed at the new temperatures) follow
 * the states; sums, sweep counters and CRBM replicas stay with the chain;
 * n_swap of both chains counts the swap.  Random numbers are indexed by r:
 * use each round index once.  Not allowed with CRBM_GIBBS. */
CRBM_API crbm_status crbm_tempering_swap(crbm_ctx* ctx, int32_t n_ladders, int32_t round);

/* Per-sweep observable trace, the input of integrated autocorrelation times
 * (the sampler diagnostic of Sec. III and IV): with trace != NULL, sweep t of
 * chain g stores the energy of the chain's state after the sweep (Ising: E/J;
 * Kitaev: the fermion energy E_f) at trace[g * trace_len + t % trace_len]
 * (device, FP64, caller-owned, [n_chains][trace_len]).  NULL or trace_len = 0
 * switches it off.  Stream-ordered like the sweeps. */
CRBM_API crbm_status crbm_set_trace(crbm_ctx* ctx, double* trace, int32_t trace_len);

/* Autocovariance and integrated autocorrelation time of n series
 * x_{g,i} = trace[g * len + (start + i) % len], i = 0..len-1 (device FP64),
 * the diagnostic by which Sec. III and IV compare samplers:
 *   out[g][t] = C(t) = 1/(len - t) sum_{i < len - t} (x_i - m)(x_{i+t} - m),
 *   m the series mean, t = 0..max_lag (device, [n][max_lag + 1]);
 *   tau[g] = 1/2 + sum_{t=1..W} C(t)/C(0) with W the smallest lag >= 1 such
 *   that W >= c_window * tau(W) (automatic windowing), window[g] = W, or -1
 *   with tau summed to max_lag when no lag qualifies or C(0) = 0.
 * tau and window (device, [n]) may both be NULL for the autocovariance alone.
 * 1 <= len <= 8176 (the series is held in 64 KiB of LDS), 0 <= max_lag < len,
 * c_window > 0.  Async on `stream`. */
CRBM_API crbm_status crbm_autocorr(const double* trace, int32_t n, int32_t len, int32_t start, int32_t max_lag,
                                   double c_window, double* out, double* tau, int32_t* window, void* stream);

/* Copy the per-chain records, n_chains x crbm_chain_stats, to `out`
 * (device memory if on_device != 0, else host memory; the host copy
 * synchronises the stream). */
CRBM_API crbm_status crbm_read_stats(crbm_ctx* ctx, crbm_chain_stats* out, int32_t on_device);

/* Sweeps done so far by the job. Host only. */
CRBM_API int64_t crbm_sweeps_done(const crbm_ctx* ctx);

/* Release the handle (host memory only; caller-owned buffers untouched). */
CRBM_API crbm_status crbm_destroy(crbm_ctx* ctx);

/* CRBM free energy, Eq. (free-energy_CRBM), of B states x[B][C][L][L] (+-1,
 * device) -> F_out[B] (device, FP64).  Terms and sums in FP64. */
CRBM_API crbm_status crbm_free_energy(const crbm_params* params, const int8_t* x, int32_t B, int32_t L,
                             double* F_out, void* stream);

/* Target of B states x[B][C][L][L] (device); boundary as in crbm_batch_desc.
 * CRBM_ISING (C must be 1): E_out[B] = E/J = -sum_<ij> s_i s_j (device int32,
 *   exact); S_out ignored (may be NULL).
 * CRBM_KITAEV (C = 1 or 3): S_out[B] = sum_lambda log 2cosh(eps_lambda/(2 T[b]))
 *   (device FP64) over the N = L^2 singular values of M; T is device [B];
 *   E_out ignored. L <= 12 for Kitaev (this op has no workspace for the
 *   larger eigen-step; jobs go to L = 24). */
CRBM_API crbm_status target_energy(int32_t target, const int8_t* x, int32_t B, int32_t C, int32_t L,
                          int32_t boundary, const double J[3] /* host */, const double* T, int32_t* E_out,
                          double* S_out, void* stream);

/* Vector-Jacobian product of F (the backward of the loss of Eq. (loss)):
 * dW = sum_b gF[b] dF(x_b)/dW, likewise dhbias, dvbias, with
 *   dF/dW[k][c][a][b'] = -sum_ij sigmoid(a[k][i][j]) v[c][(i+a)%L][(j+b')%L]
 *   dF/dhbias[k]       = -sum_ij sigmoid(a[k][i][j])
 *   dF/dvbias[c]       = -sum_ij v[c][i][j].
 * With filter banks, dW and dhbias have the banks' layout and a bank's sums
 * run over the hidden columns it owns (and, with open_cols, over the visible
 * columns inside the lattice only).
 * x[B][C][L][L] +-1 device; gF[B] float32 device; outputs float32 device,
 * overwritten.  Per-sample sums in FP32 terms / FP64 accumulation, the sum
 * over samples in FP64 in a fixed order (deterministic). `workspace` is a
 * device buffer of crbm_grad_workspace_size(params, B) bytes. */
CRBM_API size_t crbm_grad_workspace_size(const crbm_params* params, int32_t B);
CRBM_API crbm_status crbm_grad(const crbm_params* params, const int8_t* x, int32_t B, int32_t L, const float* gF,
                      float* dW, float* dhbias, float* dvbias, void* workspace, size_t workspace_bytes,
                      void* stream);

/* crbm_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, arguments and results as crbm_grad, with the per-sample
 * partial gradients in a static scratch of 8 MiB that the library holds on
 * every GPU it runs on until the process ends, instead of a caller
 * workspace.  The call allocates nothing; it needs crbm_grad_workspace_size
 * (params, B) <= 8 MiB (B * P * 8 bytes, P = banks (K C Lw^2 + K) + C, or
 * K C L^2 + K + C L^2 for a dense RBM: B <= 5017 for K = 8, Lw = 5) and
 * returns CRBM_EBUDGET beyond that, without launching.  Calls on one GPU share
 * the scratch: calls that overlap on one GPU (several streams, several host
 * threads) race; serialise them.  The device current at the call must be the
 * one the pointers and the stream belong to. */
CRBM_API crbm_status crbm_grad_static(const crbm_params* params, const int8_t* x, int32_t B, int32_t L,
                                      const float* gF, float* dW, float* dhbias, float* dvbias, void* stream);

/* Tile choice of the bit-packed Ising sweep for jobs with this (L, K, Lw):
 * `rows` lattice rows x 4 columns per lane (1, 2 or 4) and `threads` per
 * workgroup (64, 256, 512 or 1024).  Process-wide; applies to jobs created after the
 * call.  Results do not depend on the choice (random numbers are indexed by
 * unit, sweep and chain), only speed does.  Host only. */
CRBM_API crbm_status crbm_set_tuning(int32_t L, int32_t K, int32_t Lw, int32_t rows, int32_t threads);

/* Forget every tile choice (defaults apply again). Host only. */
CRBM_API crbm_status crbm_clear_tuning(void);

/* Message of the last error on the calling thread ("" if none). */
CRBM_API const char* crbm_last_error(void);

/* Version string of the library. */
CRBM_API const char* crbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CRBM_H */
