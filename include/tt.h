/*
 * tt.h -- C-ABI of the MI355X tropical tensor-network library (libtt.so).
 *
 * Problem (Eq. 1 of Liu, Wang & Zhang, "Tropical tensor network for ground
 * states of spin glasses"): E(sigma) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i
 * over sigma in {+1,-1}^n on a graph with edges (i, j). The library contracts
 * the tensor network of Sec. II (bond tensors [[J,-J],[-J,J]], field vectors
 * (h,-h), copy tensors as shared spin labels) over the max-plus semiring of
 * Eq. (2), which yields -E*; with the (x, n) tuples of Eq. (4) it also yields
 * the ground-state degeneracy g; walking the contraction backwards through
 * its argmax choices (Sec. IV) yields one ground state sigma* and the
 * gradients d(E*)/d(J_ij) = -s_i s_j and d(E*)/d(h_i) = -s_i.
 *
 * Spin encoding: index 0 <-> sigma = +1, index 1 <-> sigma = -1.
 *
 * Conventions for every call:
 *   - Return value: TT_OK (0) or a negative tt_status; the message of the
 *     last failure on the calling thread is returned by tt_last_error().
 *     No C++ exception crosses this boundary.
 *   - Arrays named "device" are device pointers on the current HIP device,
 *     owned by the caller, laid out densely as stated. Host arrays are owned
 *     by the caller and only read during the call.
 *   - Plans are owned by the library (tt_plan_destroy frees them) and may be
 *     shared by concurrent calls on different streams only if each call uses
 *     its own plan; device workspace is cached inside the plan.
 *   - Compute calls enqueue on `stream` (a hipStream_t, NULL = default
 *     stream); outputs are valid after the stream synchronises.
 *     tt_contract, tt_backward and tt_contract_uneven first check their
 *     inputs on the device (every coupling and field finite; with int32
 *     couplings sum|J| + sum|h| < 2^24 per instance, the range in which the
 *     float32 state is exact): the check is the first launch of the call, and
 *     the call returns after enqueueing all its launches and waiting for the
 *     check's result, i.e. once the work queued on `stream` before the call
 *     has finished. An input error is returned as TT_E_INVAL (not finite) or
 *     TT_E_RANGE; the outputs are then unspecified. tt_count synchronises
 *     `stream` (it checks the range and recombines the counts on the host).
 *   - An explicit budget (tt_plan_opts.max_bytes) is checked on the host
 *     before any device work: a call whose state would exceed it returns
 *     TT_E_TOOBIG without touching the device.
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tt_status {
  TT_OK = 0,
  TT_E_INVAL = -1,          /* bad graph, null pointer, bad size or option */
  TT_E_DTYPE = -2,          /* dtype not supported by this call */
  TT_E_RANGE = -3,          /* exact-integer range of the value type exceeded */
  TT_E_TOOBIG = -4,         /* planned device memory exceeds the budget */
  TT_E_COUNT_OVERFLOW = -5, /* tt_count in strict mode: g may exceed the moduli */
  TT_E_DEVICE = -6,         /* a HIP runtime call failed (message has the code) */
  TT_E_NOMEM = -7           /* host allocation failed */
} tt_status;

typedef enum tt_dtype {
  TT_F32 = 0,               /* J, h as float32; energies computed in float32 */
  TT_I32 = 1,               /* J, h as int32; computed exactly (|values| < 2^24) */
  TT_I16 = 2                /* J, h as int16; the state is held as int16 (half the bytes)
                               and worked on two entries per instruction (packed 16-bit
                               integers), exactly, for sum|J| + sum|h| < 2^13 (TT_E_RANGE
                               otherwise; Sec. V keeps the chimera state in Int16 for the
                               same reason). tt_contract, tt_backward(_tie) and
                               tt_plan_autotune on sweep and chimera plans (sliced
                               ones included); other calls return TT_E_DTYPE. A
                               backward whose pass inputs do not all fit the budget
                               recomputes them from int16 snapshots. */
} tt_dtype;

typedef enum tt_order_kind {
  TT_ORDER_GREEDY = 0,      /* host greedy search for a spin order (restarts) */
  TT_ORDER_GIVEN = 1,       /* caller's spin order (opts.order) */
  TT_ORDER_CHIMERA = 2      /* row-chain plan for a chimera graph of K_{4,4} cells */
} tt_order_kind;

/* Planner options. Zero-initialised fields take the defaults in brackets. */
typedef struct tt_plan_opts {
  int32_t kind;             /* tt_order_kind [GREEDY] */
  const int32_t* order;     /* GIVEN: permutation of 0..n-1 (host) */
  uint64_t seed;            /* GREEDY: seed of the randomised tie-breaks [0] */
  int32_t trials;           /* GREEDY: randomised restarts, the narrowest (then
                               cheapest) order kept; the restarts of one seed share
                               one random stream, so more of them never give a wider
                               plan. About 0.5 ms each at 220 spins of degree 3,
                               where thousands save two or three spins of width. [32] */
  int32_t has_field;        /* 1: instances carry fields h (else h = 0) */
  int32_t tile_bits;        /* resident bits per tile of the energy path [14] */
  int32_t count_tile_bits;  /* resident bits per tile of the count path [12] */
  int32_t chimera_rows;     /* CHIMERA: unit-cell rows  */
  int32_t chimera_cols;     /* CHIMERA: unit-cell columns */
  int64_t max_bytes;        /* device memory budget of one call [7/8 of free] */
  int32_t parts;            /* concurrent parts (streams) a large same-graph batch
                               runs in: 1 or 2 [2] */
  int32_t q;                /* labels per spin: 2 = Ising spins, 3 = 3-state Potts
                               glass (App. C; GREEDY or GIVEN order, no fields,
                               tt_potts_* calls only) [2] */
  int32_t z2;               /* 1: keep half of every energy-path state (Ising plans
                               without fields: GREEDY, GIVEN or CHIMERA order). With h = 0 Eq. (1) is
                               even under flipping every spin, and so is every partial
                               contraction: entries whose top address bit is 1 are read
                               at the complement address, and a pass runs half of its
                               tiles, each also writing its mirror outputs. Same
                               results (E*, a ground state, gradients, the exact
                               degeneracy) for about half the bytes and work of
                               every pass. tt_contract, tt_backward(_tie),
                               tt_contract_uneven(_fields) and tt_count (whose
                               (x, n) states are halved the same way) accept such
                               plans (a backward whose pass inputs do not all fit
                               recomputes them from half-size snapshots); the
                               allocation-free call returns TT_E_INVAL. [0] */
} tt_plan_opts;

typedef struct tt_plan_stats {
  int32_t n_spins;
  int64_t n_edges;
  int32_t width;            /* log2 of the largest state (entries per instance) */
  int32_t n_ops;            /* absorb/relabel/eliminate operations */
  int32_t n_passes;         /* energy-path passes (kernel launches per batch) */
  int32_t n_count_passes;   /* count-path passes */
  /* algorithmic work per instance, at the live width of every step:
   * max-plus ops = 2 * terms + elementwise; for half-state plans (z2) the
   * entries their passes visit (half of a pass's state where the pass has a
   * tile-id bit with an output position, and half of the final state) */
  double terms;             /* contraction terms (one add + one max): K per output entry */
  double elementwise;       /* elementwise ops: diagonal / field absorbs (one add per
                               entry), cuts and the final maximum (one max per entry) */
  double reduce_ops;        /* of which the final maximum over the last state */
  double entry_updates;     /* state entries read+written per instance (energy path) */
  int32_t parts;            /* concurrent parts a large same-graph batch runs in (the
                               autotuner may have chosen it) */
} tt_plan_stats;

typedef struct tt_plan tt_plan;

/* Build a contraction plan for a graph (Sec. III: order, then pairwise
 * contraction). edges: host int32 [n_edges][2], 0 <= e[0] < e[1] < n_spins,
 * no duplicates. The graph is copied. *out receives the plan. */
int tt_plan_create(int32_t n_spins, int64_t n_edges, const int32_t* edges,
                   const tt_plan_opts* opts, tt_plan** out);
/* Sliced plan: the sum of Eq. (1) split by the values of n_fixed spins, the
 * index-slicing form of the contraction (the network's largest tensors lose
 * one index per fixed spin). Each of the 2^n_fixed assignments of the fixed
 * spins (a slice) leaves an instance of the graph without them, in which a
 * bond J_ij to a fixed spin j is a field J_ij sigma_j on spin i and the bonds
 * and fields among fixed spins are a constant; E* is the minimum over the
 * slices of their energies plus constants, g the sum of the degeneracies of
 * the slices that reach it (Eq. (4)). tt_contract, tt_backward(_tie) and
 * tt_count accept sliced plans and run the slices as batches of the reduced
 * graph's plan, as many at a time as the budget (opts.max_bytes, else free
 * device memory) holds; other calls return TT_E_INVAL. tt_backward takes the
 * first minimising slice (lowest slice index, bit j of the index = fixed spin
 * j at -1) and walks it back. opts as tt_plan_create (GREEDY or GIVEN order
 * over all n_spins; has_field as for the whole graph), 1 <= n_fixed <= 16,
 * n_fixed < n_spins. fixed: host int32 [n_fixed] distinct spins, or NULL to
 * let the planner choose them (one at a time, the spin live at the most
 * points of the current sweep's largest width). tt_plan_info reports the
 * reduced plan's width and passes and the work of all slices per instance;
 * tt_plan_order the fixed spins followed by the reduced sweep's order;
 * tt_plan_ops and tt_plan_program those of the reduced plan, in its own
 * numbering (spins in ascending order without the fixed ones, edges in input
 * order without those touching a fixed spin). */
int tt_plan_create_sliced(int32_t n_spins, int64_t n_edges, const int32_t* edges,
                          const tt_plan_opts* opts, int32_t n_fixed, const int32_t* fixed,
                          tt_plan** out);
/* Number of fixed spins of a plan (0 when unsliced); fixed_out (host, may be
 * NULL) receives them, fixed index j first to last. */
int tt_plan_slice_info(const tt_plan* plan, int32_t* fixed_out);
int tt_plan_info(const tt_plan* plan, tt_plan_stats* out);
/* Host copy of the spin order the plan sweeps (n_spins int32). */
int tt_plan_order(const tt_plan* plan, int32_t* order_out);
void tt_plan_destroy(tt_plan* plan);
/* The encoded energy program the kernels execute, for host-side checks:
 * which = 0 pass descriptors, 1 stages, 2 fused ops, 3 backward candidates,
 * 4 backward terms, 5 final bit layout, 6 per pass the chimera row whose
 * chain step follows it (int32, -1 = none); for 3-state plans (opts.q = 3)
 * 7 energy passes, 8 counting passes, 9 the final-reduction descriptor;
 * for Ising plans 10 the counting path's passes, 11 its ops. Copies at most cap bytes into out
 * (may be NULL) and returns the total size in bytes (or a negative
 * tt_status). The record layouts are those of the library's device.hpp. */
int64_t tt_plan_program(const tt_plan* plan, int32_t which, void* out, int64_t cap);
/* The plan's operation list, for inspection and host-side checks: record k
 * occupies out[8k .. 8k+7] = {kind (0 INTRO, 1 GATE, 2 CUT, 3 DIAG, 4 FIELD),
 * slot_a, slot_b, param (edge for GATE/DIAG, spin for FIELD), old_spin,
 * new_spin, width_before, width_after}. Returns the number of records (or a
 * negative tt_status); writes at most cap records. final_slot_spin (may be
 * NULL) receives the spin held by each slot after the last op (-1 = free),
 * final_width entries. */
int tt_plan_ops(const tt_plan* plan, int32_t* out, int64_t cap, int32_t* final_slot_spin,
                int32_t* final_width);

/* Ground-state energy E* (Eq. 1, not its negative) of `batch` instances that
 * share the plan's graph. J: device [batch][n_edges] of dtype; h: device
 * [batch][n_spins] or NULL (required iff the plan has fields);
 * energy: device double [batch]. */
int tt_contract(tt_plan* plan, int32_t batch, int32_t dtype, const void* J,
                const void* h, double* energy, void* stream);

/* Allocation-free tt_contract, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, checks and results as tt_contract, but
 * every buffer the call needs besides the caller's inputs and outputs lives in
 * a fixed workspace of TT_NOALLOC_MAX_BYTES per GPU, part of the library's
 * device image and held until the process ends. The call makes no device
 * allocation or free (nor does any routine it calls); it launches eagerly on
 * `stream` (no graph replay, no concurrent parts) and returns after `stream`
 * has synchronised. Every call on one GPU uses that GPU's one workspace:
 * calls that overlap in time on the same GPU (other threads, other streams)
 * race and must be serialised by the caller. A batch whose state, tables and
 * partials do not fit (about batch x 2^width x 8 bytes plus a few KB) returns
 * TT_E_TOOBIG before any device work; chimera plans return TT_E_INVAL. */
#define TT_NOALLOC_MAX_BYTES (64u << 20)
int tt_contract_noalloc(tt_plan* plan, int32_t batch, int32_t dtype, const void* J,
                        const void* h, double* energy, void* stream);

/* Energy plus one ground state (Sec. IV): sigma device int8 [batch][n_spins]
 * in {+1,-1}; dJ device float [batch][n_edges] = -s_i s_j and dh device
 * float [batch][n_spins] = -s_i (either may be NULL). Ties resolve to the
 * first argument of every max along the plan. When the input of every pass
 * does not fit the budget, a same-graph sweep plan keeps as many snapshots of
 * pass inputs as fit, each the size of the widest stored state, and
 * recomputes the others segment by segment (Sec. IV: memory traded for
 * time); the results are the same bit for bit. Fewer than two such states
 * within the budget: TT_E_TOOBIG. */
int tt_backward(tt_plan* plan, int32_t batch, int32_t dtype, const void* J,
                const void* h, double* energy, int8_t* sigma, float* dJ,
                float* dh, void* stream);

/* tt_backward with a choice of tie rule (Sec. IV: max returns its first
 * argument when two are equal; other rules reach other degenerate ground
 * states): tie = 0 is tt_backward (the first maximiser at every choice), 1
 * the last, any other value a pseudo-random order per pass seeded by it. The
 * rule applies to every spin the walk chooses; spins still held by the final
 * state keep the lowest address of the final maximum. Every rule returns a
 * ground state. Sweep plans only (chimera plans: TT_E_INVAL for tie != 0). */
int tt_backward_tie(tt_plan* plan, int32_t batch, int32_t dtype, const void* J,
                    const void* h, double* energy, int8_t* sigma, float* dJ,
                    float* dh, uint64_t tie, void* stream);

/* One ground state by finite differences of E* with respect to the fields
 * (Sec. IV, the first way it names: E* is piecewise linear in h, and
 * E*(h + delta e_i) = E* - delta sigma_i while the ground state does not
 * change): the n + 1 copies of the instance (unperturbed, and h_i raised by
 * delta for each spin i) are contracted as one batch. float32 couplings and
 * fields, one instance; the plan must carry fields (h may be NULL for zero
 * fields). J: device float [n_edges]; h: device float [n_spins] or NULL;
 * energy: device double [1] = E*; sigma: device int8 [n_spins].
 * consistent (host, may be NULL; then the call does not wait): 1 when
 * Eq. (1) of sigma equals E* within 1e-5 n_spins, i.e. the ground state is
 * unique at the resolution of delta (delta must stay below half the gap to
 * the first excited state and well above the float32 rounding of E*). */
int tt_config_fd(tt_plan* plan, const float* J, const float* h, double delta,
                 double* energy, int8_t* sigma, uint8_t* consistent, void* stream);

/* A ground state drawn uniformly at random from all of them (Sec. IV, the
 * second way it names: conditional probabilities along an order of the
 * spins): for spin k = 0, 1, ... the degeneracies of the ground states with
 * the spins before it fixed as already drawn and sigma_k = +1 or -1 come from
 * the counting contraction (spins fixed by fields H > sum|J| + sum|h|), and
 * sigma_k = +1 is taken when u[k] (c+ + c-) < c+ (exact integer arithmetic
 * on the counts). int32 couplings; one instance; the plan must carry fields.
 * J: device int32 [n_edges]; h: device int32 [n_spins] or NULL; u: host
 * double [n_spins] in [0, 1) (the caller's random numbers); sigma: host int8
 * [n_spins]; energy: host int64 E*. Runs n_spins + 1 counting contractions
 * and synchronises `stream`. TT_E_RANGE when sum|J| + sum|h| + n H >= 2^24. */
int tt_sample_ground_state(tt_plan* plan, const int32_t* J, const int32_t* h,
                           const double* u, int8_t* sigma, int64_t* energy,
                           void* stream);

/* Ground-state energy and degeneracy g (Eq. 4: tuples (x, n), n an ordinary
 * count) for integer couplings. J: device int32 [batch][n_edges]; h: device
 * int32 [batch][n_spins] or NULL. energy: host int64 [batch]; residues: host
 * uint64 [batch][3], g mod the three primes of tt_count_moduli (their
 * product M ~ 2^183). g counts sigma and -sigma separately.
 * Exactness: g <= 2^n_spins, so for n_spins <= 182 the CRT value of the
 * residues is g. For larger graphs the kernels carry g mod 2^64 as well and
 * the CRT value is accepted when it agrees with it modulo 2^64 (g >= M with
 * agreement needs floor(g / M) to be a multiple of 2^64).
 * exact_flag: host uint8 [batch], 1 = the residues give g exactly, 0 = g may
 * reach M (then only g mod M is known); NULL selects strict mode, in which
 * any inexact instance makes the call return TT_E_COUNT_OVERFLOW.
 * TT_E_RANGE when sum|J| + sum|h| >= 2^24 for an instance. */
int tt_count(tt_plan* plan, int32_t batch, const int32_t* J, const int32_t* h,
             int64_t* energy, uint64_t* residues, uint8_t* exact_flag, void* stream);
/* 3-state Potts glasses (App. C): H(s) = sum_{(i,j)} J_ij M[s_i][s_j] with
 * labels s in {0, 1, 2} (the paper's 1, 2, 3) and M = 1 on the diagonal,
 * -1/2 off it. The plan comes from tt_plan_create with opts.q = 3 (GREEDY or
 * GIVEN order, no fields); its state has 3^width entries per instance
 * (width <= 20). The contraction runs over doubled energies 2H, exact for
 * integer couplings while 2 sum|J| < 2^24 (else TT_E_RANGE).
 *
 * tt_potts_contract: ground-state energy H* (a multiple of 1/2 for integer
 * couplings) of `batch` (<= 65535) instances sharing the plan's graph.
 * J: device [batch][n_edges] float32 or int32 (dtype); energy: device double
 * [batch]. Inputs are checked on the device like tt_contract's (TT_E_INVAL
 * for a non-finite coupling, TT_E_RANGE). */
int tt_potts_contract(tt_plan* plan, int32_t batch, int32_t dtype, const void* J,
                      double* energy, void* stream);
/* tt_potts_count: ground-state energy and degeneracy g (Eq. 4 tuples) for
 * int32 couplings. energy2: host int64 [batch] = 2H*; residues: host uint64
 * [batch][3], g modulo the primes of tt_count_moduli; g counts labelings, so
 * it is a multiple of 3 (label permutations). g <= 3^n_spins: exact for
 * n_spins <= 115; beyond, a plane modulo 2^64 checks the CRT value as in
 * tt_count (exact_flag: host uint8 [batch], 1 = exact; NULL = strict mode,
 * TT_E_COUNT_OVERFLOW). Synchronises `stream`. */
int tt_potts_count(tt_plan* plan, int32_t batch, const int32_t* J, int64_t* energy2,
                   uint64_t* residues, uint8_t* exact_flag, void* stream);

/* The three prime moduli (2^61-1, 2^61-31, 2^61-45). */
int tt_count_moduli(uint64_t moduli_out[3]);
/* Exact g from its residues by the Chinese remainder theorem, as a decimal
 * string (host). Exact whenever g < the product of the moduli (~2^183). */
int tt_count_to_decimal(const uint64_t residues[3], char* buf, size_t len);

/* Natural logarithm of g from its residues (for the residual entropy
 * s = ln g / n_spins of Sec. V), from the exact CRT value; relative error
 * below 1e-15. TT_E_INVAL for g = 0 or unreduced residues. */
int tt_count_log(const uint64_t residues[3], double* log_g);

/* Uneven batch: n_inst instances, each with its own plan, contracted forward
 * and backward together (one launch per pass index across instances).
 * J: device float/int32 concatenated, instance i at j_off[i] (host int64);
 * sigma: device int8 concatenated at s_off[i] (host int64) (may be NULL);
 * dJ: device float laid out like J (may be NULL); energy: device double
 * [n_inst]. Every plan must be without fields (see tt_contract_uneven_fields). */
int tt_contract_uneven(int32_t n_inst, tt_plan* const* plans, int32_t dtype,
                       const void* J, const int64_t* j_off, double* energy,
                       int8_t* sigma, const int64_t* s_off, float* dJ,
                       void* stream);
/* tt_contract_uneven with fields: instance i's fields (of J's dtype) at
 * h + h_off[i] when plans[i] carries fields (h_off[i] is ignored otherwise);
 * dh (may be NULL; needs sigma) laid out like h receives -sigma_i for the
 * instances with fields. h may be NULL when no plan carries fields. */
int tt_contract_uneven_fields(int32_t n_inst, tt_plan* const* plans, int32_t dtype,
                              const void* J, const int64_t* j_off, const void* h,
                              const int64_t* h_off, double* energy, int8_t* sigma,
                              const int64_t* s_off, float* dJ, float* dh,
                              void* stream);

/* Dense tropical matrix product (Eq. 2 as a matrix product, the contraction
 * of two tensors over a run of shared labels):
 *   C[b][i][j] = max_k (A[b][i][k] + B[b][k][j]),  b < batch.
 * A, B, C: device float32, row-major with leading dimensions lda, ldb, ldc
 * (elements) and batch strides sA, sB, sC (elements). K = 0 gives -inf.
 * Each term is one float32 add; max is exact, so C equals the float64
 * product rounded to float32. */
int tt_tgemm(int32_t batch, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, int64_t sA,
             const float* B, int64_t ldb, int64_t sB, float* C, int64_t ldc, int64_t sC, void* stream);

/* HIP-graph replay of repeated calls (on by default): tt_contract,
 * tt_backward and tt_contract_uneven calls whose plans, sizes and device
 * addresses equal those of an earlier call are captured once (on their
 * second occurrence) and then replayed as one graph launch on an internal
 * stream, ordered after and before `stream` by events. A replay reads the
 * current contents of the inputs, so it is equivalent to the eager call.
 * Large same-graph batches (batch * 2^width >= 2^20 state entries) are never
 * captured: they run eagerly in two parts, the first on `stream` and the
 * second on an internal stream forked from and joined to `stream` by events
 * (the call is ordered on `stream` like any other). */
int tt_graphs_enable(int32_t on);

/* Tile-size autotuner (batched execution, tiles chosen per plan): times the
 * call the tiles will serve, on `batch` instances given as for that call, on
 * `stream`, and keeps the fastest tile size in the plan for later calls.
 * mode: TT_TUNE_ENERGY times tt_contract (tiles of up to 14 bits),
 * TT_TUNE_COUNT tt_count (up to 12 bits; int32 couplings), TT_TUNE_BACKWARD
 * tt_backward (energy, one configuration and both gradients; the backward
 * sweep's cost grows with the spins a pass eliminates, so it can prefer
 * smaller tiles than the energy alone). Candidates: the five sizes below the
 * largest useful one (min(maximum, state width)), never under 7 bits. The
 * score is the summed device time of the call's kernels, the least of three
 * calls; for a same-graph batch of at least 2^20 state entries (which runs in
 * parts on concurrent streams) it is the device time from before to after the
 * call instead, and when the plan left the part count to the library
 * (tt_plan_opts.parts = 0) every tile size is also timed in one part and the
 * faster count is kept (tt_plan_info reports it). Blocks until the timing is done; allocates the timed calls' outputs
 * (freed before it returns). chosen_bits and best_ms (milliseconds per call)
 * may be NULL. Captured graphs and device buffers of the plan are released.
 * TT_E_INVAL for an unknown mode. */
enum { TT_TUNE_ENERGY = 0, TT_TUNE_COUNT = 1, TT_TUNE_BACKWARD = 2 };
int tt_plan_autotune(tt_plan* plan, int32_t batch, int32_t dtype, const void* J, const void* h, int32_t mode,
                     int32_t* chosen_bits, double* best_ms, void* stream);

/* Per-kernel timing on the call's stream, for measurement tools: when on,
 * every launch is bracketed by HIP events (the pass kernel's two events are
 * handed to its launch, which stamps them with the kernel's own start and
 * end, dispatch excluded) and calls run eagerly (no graph
 * capture or replay); tt_prof_read returns the summed milliseconds and
 * launch count of the named kernel family ("sweep_pass", "sweep_backward",
 * "final_reduce", "count_pass", "count_reduce", "count_chain", "chain",
 * "row_argmax", "chimera_finish", "tgemm", "check_inputs", "potts_pass",
 * "potts_reduce", "potts_count_pass", "potts_count_reduce") since the last reset. Timing adds
 * no work to the launches themselves. */
int tt_prof_enable(int32_t on);
int tt_prof_reset(void);
int tt_prof_read(const char* name, double* total_ms, int64_t* launches);

/* Thread-local message of the last failure ("" if none). */
const char* tt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TT_H */
