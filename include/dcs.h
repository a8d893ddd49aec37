/*
 * dcs.h - C ABI of the MI355X (gfx950) library for number-conserving sectors:
 * the divide-and-conquer basis index and the matrix-free product y = H x.
 *
 * The method is that of R. Schaefer and D. J. Luitz, "DanceQ: High-performance
 * library for number-conserving bases", SciPost Phys. Codebases 48 (2025),
 * arXiv:2407.14591.  Section references below are to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - A sector is the set of product states of L sites with Q states each
 *    (digits 0..Q-1) whose digit sum is n (Sec. 2.1).  Its states are numbered
 *    0..D-1 in the canonical order of Sec. 3.1-3.2: the sites are cut into
 *    subsystems P_0..P_{N-1} (consecutive sites, P_0 first); P_0 varies
 *    slowest; inside a subsystem, words are grouped by their digit sum (lower
 *    first) and ordered lexicographically (first site most significant).
 *  - State encoding (Sec. 4.2): one uint64_t per state, ceil(log2 Q) bits per
 *    site, site 0 in the most significant field of the low L*ceil(log2 Q)
 *    bits, plain binary digits.  Bits above that must be zero.
 *  - Pointers named d_* are device pointers on the sector's device; h_* are
 *    host pointers.  The caller owns every pointer it passes; the library
 *    owns only the objects it creates (their tables live on the device).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls that take a
 *    stream only enqueue work on it and return; results are ready when the
 *    stream is synchronised.  Calls without a stream may synchronise.
 *  - Every call returns DCS_OK (0) or a negative status; dcs_last_error()
 *    gives a message for the last failing call of the calling thread.  No
 *    exception crosses the ABI.  A kernel fault surfaces at the caller's next
 *    synchronisation of the stream.
 *  - Index type: indices are uint64_t in the ABI.  Sectors with D < 2^32 - 1 run
 *    their kernels with 32-bit index arithmetic; larger ones with 64-bit.  The
 *    environment variable DCS_INDEX_BITS=64, read by dcs_sector_create, forces
 *    64-bit arithmetic (to test those kernels on small sectors).
 *  - Split product: for Q = 2 sectors with at least 2^20 states and two or
 *    more subsystems, dcs_sector_create also builds a left/right view (cut after
 *    N/2 subsystems: every left configuration owns a contiguous run of rows, one
 *    per right configuration).  The first dcs_hamiltonian_apply with a terms
 *    object builds that pair's target tables (host work, then kept with the
 *    sector for the next calls; up to four terms objects per sector) and every
 *    product runs three kernels: the diagonal per configuration of each side,
 *    one pass over the rows for the bonds right of and across the cut, and one
 *    over column chunks for the bonds left of it (or, in the fused form, two:
 *    the row pass also applies the bonds left of the cut).  Target offsets
 *    inside a run are 16-bit for runs below 65,535 rows and 32-bit for longer
 *    runs (up to 2^25 rows; beyond that the single pass runs).  DCS_SPLIT_MIN_DIM
 *    (read by dcs_sector_create) changes the 2^20 threshold; DCS_SPLIT=0 (read
 *    at every product) forces the single pass; DCS_SPLIT_LDS=0 (likewise) keeps
 *    the row pass from staging runs of x in on-chip memory; DCS_SPLIT_FUSED=1
 *    (likewise) makes the fused form the default form, DCS_SPLIT_TILED=1 the
 *    block-tiled one (DCS_FORM_SPLIT_TILED).
 */
#ifndef DCS_H
#define DCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define DCS_OK 0
#define DCS_EINVAL (-1)       /* bad argument */
#define DCS_ERANGE (-2)       /* index range past the end of the sector */
#define DCS_ENOMEM (-3)       /* device or host allocation failed */
#define DCS_EHIP (-4)         /* a HIP runtime call failed (message has the HIP error) */
#define DCS_EUNSUPPORTED (-5) /* valid but beyond this build's limits (message says which) */

/* ---- element types of vectors ------------------------------------------- */
#define DCS_F32 0
#define DCS_F64 1
#define DCS_C64 2  /* complex, interleaved FP32 (re, im) pairs (generic operators only) */
#define DCS_C128 3 /* complex, interleaved FP64 (re, im) pairs (generic operators only) */

/* ---- Lanczos re-orthogonalisation modes --------------------------------- */
#define DCS_REORTH_NONE 0  /* plain three-term recurrence */
#define DCS_REORTH_LOCAL 1 /* exact projection out of span(v_{j-1}, v_j) each step */
#define DCS_REORTH_FULL 2  /* two classical Gram-Schmidt passes against all v_0..v_j */

#define DCS_INVALID_INDEX UINT64_MAX /* rank of an invalid state, unrank of an index >= D */

/* Limits of this build */
#define DCS_MAX_SITES 64
#define DCS_MAX_SUBSYSTEMS 8
#define DCS_MAX_BONDS 256

typedef struct dcs_sector dcs_sector;
typedef struct dcs_terms dcs_terms;
typedef struct dcs_plan dcs_plan;

/* Message for the last failing call on this thread ("" if none).  The string
 * stays valid until the next library call on the same thread. */
const char *dcs_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int dcs_version(void);

/* ========================================================================== */
/* Sector: the basis with its divide-and-conquer index (Sec. 3.2, 4.2)        */
/* ========================================================================== */

/*
 * Build the index of the sector (L sites, local dimension Q = local_dim,
 * digit sum n = n_particles) cut into num_subsystems consecutive parts of
 * sizes[0..N-1] sites (P_0 first).  sizes == NULL selects the most-equal
 * split into ceil(L / floor(9 / ceil(log2 Q))) parts, shorter parts first.
 *
 * The host computes the sector dimension D_Q (App. A), the offsets and strides
 * of eq. offset / eq. stride for every (subsystem, lambda, n_k), and the local
 * lookup tables (Sec. 4.2, memory-aligned list, lexicographic inside each
 * digit sum), then copies them to `device`.  The returned object owns them.
 *
 * Table placement (Sec. 4.2 containers, Sec. 4.3 choice of N): tables of at
 * most 112 KiB are copied into LDS by every kernel that reads them; larger
 * tables (for instance the 16/16 and 10/11/11 splits of L = 32) stay in device
 * memory and are read through the caches (DCS_GLOBAL_TABLES=1 in the
 * environment at creation forces this placement).  With tables in device memory,
 * rank, unrank, enumerate, the split product (Q = 2), the one-pass product of one
 * column and the adjoint of one column work as usual; the one-pass product and the
 * adjoint of a block of k > 1 columns need the tables in LDS (such a block product
 * runs only on the split tables, else DCS_EUNSUPPORTED), and dcs_plan_create
 * rejects such a sector unless it has a split view (which runs its own product).
 *
 * Errors: DCS_EINVAL if Q < 2, L < 1, L*ceil(log2 Q) > 64, n outside
 * [0, (Q-1)L], sizes not positive or not summing to L; DCS_EUNSUPPORTED if
 * N > DCS_MAX_SUBSYSTEMS, a subsystem word wider than 16 bits, or a subsystem
 * with more than 2^14 words of one digit sum (the decode's quotient bound);
 * DCS_ENOMEM / DCS_EHIP on allocation.
 */
int dcs_sector_create(int L, int n_particles, int local_dim, int num_subsystems,
                      const int *sizes, int device, dcs_sector **out);

/*
 * The same with a local dimension per site (Sec. 5 names sites of different Q,
 * such as mixed spins, as a direct generalisation): site i has local_dims[i]
 * states in [2, 16]; the digits are packed ceil(log2 max_i local_dims[i]) bits
 * per site, and a state whose digit on site i is >= local_dims[i] is outside the
 * sector (rank gives the sentinel).  Every count of the index becomes a product
 * over the sites' own (1 + x + ... + x^{q_i - 1}) (App. A), each subsystem's
 * words are those with valid digits, and the offsets, strides and bounds of
 * eq. offset / eq. stride follow from them; rank, unrank, enumerate, the
 * sorted-list rank and the generic operators (dcs_operator_create_mixed) work
 * on such a sector.  The XXZ products (dcs_hamiltonian_apply and its adjoint,
 * expectation values, plans, dcs_lanczos) take one local dimension on every site
 * and return DCS_EUNSUPPORTED for a sector with several.  A list with one value
 * everywhere gives the same sector as dcs_sector_create.  Errors as there, with
 * n outside [0, sum_i (local_dims[i] - 1)], and DCS_EINVAL for a NULL list.
 */
int dcs_sector_create_mixed(int L, int n_particles, const int32_t *local_dims, int num_subsystems,
                            const int *sizes, int device, dcs_sector **out);

/* The local dimension of every site (L entries). */
int dcs_sector_local_dims(const dcs_sector *sector, int32_t *local_dims);

/* Free the sector's device tables and the object.  NULL is accepted. */
int dcs_sector_destroy(dcs_sector *sector);

/* Exact sector dimension D_Q(L, n) (eq. dim). */
int dcs_sector_dim(const dcs_sector *sector, uint64_t *dim);

/* Number of subsystems and their sizes (sizes may be NULL; else >= N entries). */
int dcs_sector_split(const dcs_sector *sector, int *num_subsystems, int *sizes);

/* Placement of the sector's index tables (see dcs_sector_create): *in_device_memory
 * is 1 when kernels read them in device memory, 0 when they stage them in LDS;
 * *bytes is their size.  Either output may be NULL. */
int dcs_sector_tables(const dcs_sector *sector, int *in_device_memory, size_t *bytes);

/*
 * Batched rank, function (i) of Sec. 2.2 / Alg. i: d_idx[t] = index of
 * d_states[t] = sum_k offset_k(n_k, lambda_k) + stride_k(n_k, lambda_k) * index_k
 * (eq. index, eq. ck).  A state that is not in the sector (a digit >= Q, bits
 * above L*ceil(log2 Q), or the wrong digit sum) gets DCS_INVALID_INDEX and, if
 * d_num_invalid != NULL, is added to *d_num_invalid (a device counter that the
 * call increments, not clears).  count == 0 is a no-op.  d_states and d_idx
 * must not overlap.
 */
int dcs_rank(const dcs_sector *sector, const uint64_t *d_states, uint64_t *d_idx, size_t count,
             uint64_t *d_num_invalid, void *stream);

/*
 * dcs_rank with the subsystem lookup kept as container (ii) of Sec. 4.2 instead of
 * (i): each subsystem's index comes from a binary search for its word among the
 * valid words of the same digit sum, stored in lexicographic order (the sector's
 * inverse tables, D_Q(L_k, m) entries per digit sum m), not from the table indexed
 * by the word's integer value (2^(L_k ceil(log2 Q)) entries); then eq. ck as
 * dcs_rank.  Same results, invalid states and counting as dcs_rank; for comparing
 * the containers on the device.
 */
int dcs_rank_search(const dcs_sector *sector, const uint64_t *d_states, uint64_t *d_idx,
                    size_t count, uint64_t *d_num_invalid, void *stream);

/*
 * Batched unrank, function (iii) of Sec. 2.2 / Alg. iii: d_states[t] = the state
 * with index d_idx[t].  Indices >= D give DCS_INVALID_INDEX (as a state value)
 * and are counted like dcs_rank's invalid states.
 */
int dcs_unrank(const dcs_sector *sector, const uint64_t *d_idx, uint64_t *d_states, size_t count,
               uint64_t *d_num_invalid, void *stream);

/*
 * Rank and unrank without tables of states, for spin-1/2 (Q = 2) sectors of L sites
 * and n particles cut into L single-site subsystems (eq. N=L): the canonical order is
 * then the lexicographic order of the site strings, site 0 first (the numeric order of
 * the packed states), and Alg. on-the-fly gives the rank as the sum over occupied
 * sites i of C(L-1-i, n - lambda_i).  No sector object and no stored tables: every
 * workgroup derives the binomials it needs (L rows of n + 1 counts) in LDS by App. A's
 * recurrence before serving its states (the paper's on-the-fly limit, the counterpart
 * of the table containers in the split sweep).  The same kernels serve any Q
 * (dcs_lex_rank_q) and per-site dimensions (dcs_lex_rank_mixed).  States, indices,
 * invalid entries and counting as dcs_rank / dcs_unrank.  DCS_EINVAL for L outside
 * [1, 64] or n outside [0, L].
 */
int dcs_lex_rank(int L, int n_particles, const uint64_t *d_states, uint64_t *d_idx, size_t count,
                 uint64_t *d_num_invalid, void *stream);
int dcs_lex_unrank(int L, int n_particles, const uint64_t *d_idx, uint64_t *d_states, size_t count,
                   uint64_t *d_num_invalid, void *stream);

/*
 * The same for any local dimension Q in [2, 16] (eq. N=L with D_Q): the canonical
 * order of L single-site subsystems is the lexicographic order of the digit strings
 * (ceil(log2 Q) bits per site, site 0 most significant), and Alg. on-the-fly gives
 * the rank as the sum over the sites i of sum_{k < q_i} D_Q(L-1-i, n - lambda_i - k).
 * No sector object and no tables of states: every workgroup derives the counts
 * D_Q(g, m), g < L, m <= n, in LDS by App. A's recurrence before serving its states,
 * and unrank walks them digit by digit.  States with a digit >= Q, set bits above the
 * L fields or another digit sum rank to DCS_INVALID_INDEX; indices >= D unrank to it;
 * both are counted as in dcs_rank.  DCS_EINVAL for Q outside [2, 16], L < 1 or
 * L ceil(log2 Q) > 64, n outside [0, (Q-1) L]; DCS_EUNSUPPORTED if a count reaches
 * 2^64 or the count table passes 64 KiB of LDS.
 */
int dcs_lex_rank_q(int L, int n_particles, int Q, const uint64_t *d_states, uint64_t *d_idx, size_t count,
                   uint64_t *d_num_invalid, void *stream);
int dcs_lex_unrank_q(int L, int n_particles, int Q, const uint64_t *d_idx, uint64_t *d_states, size_t count,
                     uint64_t *d_num_invalid, void *stream);

/* The same with a local dimension per site (Sec. 5's generalisation; local_dims: L
 * host entries in [2, 16], digits packed ceil(log2 max) bits per site): the counts
 * become those of the last g sites with their own dimensions, and a digit at or above
 * its site's dimension is invalid.  Errors as dcs_lex_rank_q, DCS_EINVAL for a NULL
 * list or n outside [0, sum_i (local_dims[i] - 1)]. */
int dcs_lex_rank_mixed(int L, int n_particles, const int32_t *local_dims, const uint64_t *d_states,
                       uint64_t *d_idx, size_t count, uint64_t *d_num_invalid, void *stream);
int dcs_lex_unrank_mixed(int L, int n_particles, const int32_t *local_dims, const uint64_t *d_idx,
                         uint64_t *d_states, size_t count, uint64_t *d_num_invalid, void *stream);

/*
 * Enumeration, function (ii) of Sec. 2.2 applied count-1 times from state
 * `first`: d_states[t] = state with index first + t.  Does not wrap: returns
 * DCS_ERANGE if first + count > D (the paper's increment wraps to the first
 * state; a range past the end is an error here).
 */
int dcs_enumerate(const dcs_sector *sector, uint64_t first, size_t count, uint64_t *d_states,
                  void *stream);

/* ========================================================================== */
/* Terms: the bond topology of an XXZ Hamiltonian                             */
/* ========================================================================== */

/*
 * H = sum_b [ Jxy_b/2 (S+_i S-_j + S-_i S+_j) + Jz_b Sz_i Sz_j ] + sum_i h_i Sz_i
 * (eq. H_30 and App. D, with per-bond couplings), spin S = (Q-1)/2, Sz = d - S
 * for digit d.  This object holds the topology only: bond b joins sites
 * site_i[b] != site_j[b] (host arrays, copied).  The couplings are passed to
 * every apply call, so they can change without rebuilding anything.
 *
 * Errors: DCS_EINVAL for num_bonds < 0, a negative site, site_i == site_j;
 * DCS_EUNSUPPORTED for num_bonds > DCS_MAX_BONDS or a site >= DCS_MAX_SITES.
 */
int dcs_terms_create(int num_bonds, const int32_t *site_i, const int32_t *site_j,
                     dcs_terms **out);
int dcs_terms_destroy(dcs_terms *terms);

/* ========================================================================== */
/* Matrix-free product (Sec. 2.2, Sec. 4.4)                                   */
/* ========================================================================== */

/*
 * Y = H X on the sector, X and Y of shape [D][k] row-major (k contiguous
 * columns per basis state), element type dtype (DCS_F32 or DCS_F64), k in
 * {1, 2, 4, 8}.  d_jxy and d_jz hold num_bonds FP64 couplings (device); d_h
 * holds L FP64 fields or is NULL.  Each output row is computed by one thread
 * from the row's state (pull: H is real symmetric), so Y is written once,
 * with no atomics, and the result is bitwise reproducible.  X and Y must not
 * overlap.  All bond sites must be < L.
 * Arithmetic: products and sums in dtype; couplings rounded to dtype.
 * Calls on one sector must not overlap in time (they share the sector's tile
 * counters and its cached split tables).  On a sector with a split view the
 * first call with a terms object builds that pair's tables on the host and
 * allocates them on the device (see "Split product" above); later calls
 * allocate nothing.  Autotuner: the first call for a (terms, dtype, k) on a
 * sector with a split view also times the launch forms (split product with
 * runs staged in on-chip memory, split product without, fused split product,
 * single pass; each twice, HIP events, synchronising the stream), keeps the
 * fastest for that key and returns its Y; later calls use it.  Inside stream
 * capture, or with DCS_AUTOTUNE=0 in the environment, the default form (staged
 * split, or fused with DCS_SPLIT_FUSED=1) is used.
 */
int dcs_hamiltonian_apply(const dcs_sector *sector, const dcs_terms *terms, const double *d_jxy,
                          const double *d_jz, const double *d_h, int dtype, int k,
                          const void *d_x, void *d_y, void *stream);

/* Launch forms of a product (see dcs_hamiltonian_apply). */
#define DCS_FORM_UNTUNED (-1)      /* split view, but no product of this key has run yet */
#define DCS_FORM_SPLIT_STAGED 0    /* split product, runs staged in on-chip memory where they fit */
#define DCS_FORM_SPLIT_GLOBAL 1    /* split product, row pass reading the runs from memory */
#define DCS_FORM_SPLIT_FUSED 2     /* split product whose row pass also applies the left family */
#define DCS_FORM_SINGLE 3          /* one pass with per-row decode and incremental ranks */
#define DCS_FORM_SPLIT_TILED 4     /* split product whose row pass stages whole particle-number
                                      blocks of a run in on-chip memory (rows of 16 to 64 bytes) */

/*
 * The launch form that dcs_hamiltonian_apply uses for (terms, dtype, k) on the
 * sector: the form the autotuner kept, DCS_FORM_UNTUNED before the first
 * product of that key (with the autotuner on), the default form with the
 * autotuner off (DCS_AUTOTUNE=0), DCS_FORM_SINGLE where the sector has no split
 * view, the split is switched off (DCS_SPLIT=0) or its tables do not apply.
 * Host only: reads the sector's record, launches nothing, builds nothing.
 */
int dcs_hamiltonian_form(const dcs_sector *sector, const dcs_terms *terms, int dtype, int k,
                         int *form);

/*
 * Workspace bytes that dcs_hamiltonian_apply_adjoint needs for this pair and
 * blocks of k columns (k in {1, 2, 4, 8}).  For k > 1 a smaller workspace (the
 * size for k = 1) is accepted and then rules out the split-table way.
 */
int dcs_adjoint_workspace_size(const dcs_sector *sector, const dcs_terms *terms, int k,
                               size_t *bytes);

/*
 * Fused backward of y = H(theta) X for an upstream gradient G, X and G of shape
 * [D][k] row-major (k in {1, 2, 4, 8}, as dcs_hamiltonian_apply):
 *   d_grad_x[s][c]  = (H G)_{s,c}                     (H^T = H)
 *   d_grad_jxy[b]   = sum_{s,c} G_{s,c} ((S+_i S-_j + S-_i S+_j)/2 X)_{s,c}
 *   d_grad_jz[b]    = sum_{s,c} G_{s,c} (Sz_i Sz_j X)_{s,c}
 *   d_grad_h[i]     = sum_{s,c} G_{s,c} (Sz_i X)_{s,c}    (skipped if d_grad_h == NULL)
 * For k = 1 three ways compute it: (0) one fused pass that ranks every reached
 * state once and uses it for both g and x; on a sector with a split view whose
 * products run on the split tables (the form the autotuner keeps for this terms
 * object and dtype at k = 1, see dcs_hamiltonian_apply, including its first-call
 * timing), (1) d_grad_x from that product applied to g and a pass forming only
 * the sums (it gathers x, not g), and for FP32 (2) the sums formed inside the
 * split product of g itself: each hop's gathered g_t times x at the row gives the
 * coupling sum (the hop is symmetric), and per-run / per-right-configuration sums
 * of x_s g_s give the S^z S^z and field sums.  For k > 1 two ways: (1) d_grad_x
 * from the block product H G (dcs_hamiltonian_apply, the same form) and one pass
 * over the rows that ranks every reached state and dots the k columns of X and G
 * at every hop; and for FP32 on a split view (2) the sums formed inside the split
 * block product of G as for k = 1, each hop's value the dot of the k gathered
 * columns of G with the k columns of X at the row.  The first call for a
 * (terms, dtype, k) times the ways
 * that apply (each twice, HIP events, synchronising the stream) and keeps the
 * fastest (way 2 where it applies, else 1, inside stream capture or with
 * DCS_AUTOTUNE=0; DCS_ADJOINT_WAY=0/1/2 in the environment forces a way).  The
 * sums are reduced per workgroup or per tile into d_workspace and then in a
 * fixed order, so the result is deterministic.  The coupling gradients are
 * FP64 whatever dtype is.  d_grad_x may be NULL (only coupling gradients);
 * it must not overlap d_x or d_g (DCS_EINVAL).
 */
int dcs_hamiltonian_apply_adjoint(const dcs_sector *sector, const dcs_terms *terms,
                                  const double *d_jxy, const double *d_jz, const double *d_h,
                                  int dtype, int k, const void *d_x, const void *d_g, void *d_grad_x,
                                  double *d_grad_jxy, double *d_grad_jz, double *d_grad_h,
                                  void *d_workspace, size_t workspace_bytes, void *stream);

/*
 * The adjoint above without a workspace, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and results as
 * dcs_hamiltonian_apply_adjoint minus (d_workspace, workspace_bytes); always the
 * fused single pass (it builds no split tables and times no launch forms, so
 * d_grad_x may differ from the other entry point's by rounding in FP32; the
 * coupling sums are the same).  The per-workgroup partial sums go to a fixed
 * 4 MiB device array of the library, one per GPU, kept until the process ends;
 * the call returns DCS_EUNSUPPORTED when the single pass needs more than 4 MiB
 * of partial sums (one row of 2 * num_bonds + L doubles per workgroup).  It calls no allocating routine.  Every call on one GPU shares that
 * array, so calls that overlap in time on one GPU (other streams, other
 * threads) race and must be serialised by the caller.
 */
int dcs_hamiltonian_apply_adjoint_noalloc(const dcs_sector *sector, const dcs_terms *terms,
                                          const double *d_jxy, const double *d_jz,
                                          const double *d_h, int dtype, const void *d_x,
                                          const void *d_g, void *d_grad_x, double *d_grad_jxy,
                                          double *d_grad_jz, double *d_grad_h, void *stream);

/*
 * Expectation values of the terms of H (App. D's observables) in num real
 * states psi_e (device, vec_dtype, D elements each, state e at d_psi + e*D):
 *   d_exy[e*B + b] = psi_e^T ((S+_i S-_j + S-_i S+_j)/2) psi_e
 *   d_ez [e*B + b] = psi_e^T (Sz_i Sz_j) psi_e                (bond b = (i, j), B bonds)
 *   d_esz[e*L + i] = psi_e^T Sz_i psi_e                        (skipped if NULL)
 * (device FP64 outputs).  The states are not normalised by the call: for a
 * state of norm r the values are r^2 times the expectation.  <H> for couplings
 * theta is sum_b (jxy_b exy_b + jz_b ez_b) + sum_i h_i esz_i.  Each value is
 * the adjoint's coupling sum for that term with g = x = psi_e (the sums-only
 * fused pass, one launch per state, deterministic).  d_workspace: at least
 * dcs_expectation_workspace_size bytes.
 */
int dcs_expectation_workspace_size(const dcs_sector *sector, const dcs_terms *terms,
                                   size_t *bytes);
int dcs_expectation_values(const dcs_sector *sector, const dcs_terms *terms, int vec_dtype,
                           int num, const void *d_psi, double *d_exy, double *d_ez,
                           double *d_esz, void *d_workspace, size_t workspace_bytes,
                           void *stream);

/* ========================================================================== */
/* Generic local operators (Sec. 4.1 operator strings; App. C clusters)      */
/* ========================================================================== */

typedef struct dcs_operator dcs_operator;

/*
 * O = sum_t coef_t M_t, the operator class of Sec. 4.1: each term acts on the
 * m_t = term_nsites[t] sites listed in term_sites (concatenated over the terms,
 * sites distinct, in [0, L)) with a Q^m x Q^m matrix <b|M|a> in term_mats
 * (concatenated, row-major: row = output; real, or with complex_mats = 1 complex
 * as interleaved (re, im) doubles: Sec. 4.1's scalar type), the local index of a digit string
 * (d_0, .., d_{m-1}) over the listed sites being sum_j d_j Q^(m-1-j) (the first
 * listed site most significant).  An operator string such as S+_i S-_j is the
 * Kronecker product of its single-site matrices; a custom local operator is any
 * such matrix.  The sum of the terms merged into each cluster (below) must
 * conserve the particle number, so that O maps each U(1) sector into itself:
 * its entries that join digit strings of different digit sums must cancel (to
 * 1e-13 of the cluster's largest entry; they are then dropped), else DCS_EINVAL
 * names the cluster.  A single term need not conserve (Sx Sx and Sy Sy on one
 * bond do not, their sum does) as long as the terms that restore it share its
 * cluster.
 *
 * As in App. C, the terms are merged into clusters of sites: in the given order
 * a term joins the first cluster whose site set, extended by the term's sites,
 * has at most cluster_sites sites (1..8) and Q^sites <= 4096, else it opens a new
 * cluster.  Each cluster's summed matrix is stored sparse, row by row, with the
 * packed input digits and the value (FP64 and FP32 copies, complex for a complex
 * operator) of every nonzero,
 * in device memory of `device` (owned by the object, freed by destroy).
 * Limits: 1..8 sites and Q^m <= 4096 per term (DCS_EUNSUPPORTED), Q in [2, 16],
 * L in [1, DCS_MAX_SITES].  Checks run before any device call.  Host call.
 */
int dcs_operator_create(int Q, int L, int num_terms, const int32_t *term_nsites,
                        const int32_t *term_sites, const double *term_coefs,
                        const double *term_mats, int complex_mats, int cluster_sites,
                        int device, dcs_operator **out);

/*
 * The same on sites of different local dimensions (Sec. 5's generalisation; the
 * sectors of dcs_sector_create_mixed): site i has local_dims[i] states, a term's
 * matrix has one row and one column per digit string on its sites (the product
 * of their dimensions, <= 4096, as is a cluster's), and the local index of
 * (d_0, .., d_{m-1}) is the mixed-radix number with the first listed site most
 * significant.  dcs_operator_apply requires the sector's local dimensions to match
 * site by site (DCS_EINVAL).  Errors as dcs_operator_create.
 */
int dcs_operator_create_mixed(int L, const int32_t *local_dims, int num_terms, const int32_t *term_nsites,
                              const int32_t *term_sites, const double *term_coefs,
                              const double *term_mats, int complex_mats, int cluster_sites,
                              int device, dcs_operator **out);
int dcs_operator_destroy(dcs_operator *op);

/* Clusters, stored nonzeros, the largest cluster's site count, and whether the stored
 * values are complex (any output may be NULL).  Complex terms whose merged sums are
 * real (imaginary parts within 1e-13 of the largest entry, e.g. Sx Sx + Sy Sy) give
 * a real operator. */
int dcs_operator_info(const dcs_operator *op, int *num_clusters, uint64_t *nnz,
                      int *max_cluster_sites, int *is_complex);

/*
 * d_y = O d_x on one sector (Q and L of the operator, same device): d_x, d_y of
 * D rows of dtype, DCS_F32 / DCS_F64 for a real operator, DCS_C64 / DCS_C128
 * (interleaved re, im) for a real or a complex one (a complex operator on real
 * vectors is DCS_EINVAL); the stored values are rounded to FP32 for the FP32
 * types.  Real vectors may be blocks of k columns, [D][k] row-major with k in
 * {1, 2, 4, 8} (one unrank and one rank per reached state serve all k); complex
 * vectors take k = 1 (else DCS_EUNSUPPORTED).  Pull form: one thread per row s unranks s (Alg. iii), and per cluster
 * reads s's digits on the cluster's sites (packed nb bits per site, the row
 * key), walks that row of the cluster
 * matrix, writes each entry's digits into s, ranks the result (eq. index; a
 * diagonal entry keeps s) and accumulates value * x there.  d_y must not overlap
 * d_x (DCS_EINVAL).  Asynchronous on `stream`.
 */
int dcs_operator_apply(const dcs_sector *sector, const dcs_operator *op, int dtype, int k,
                       const void *d_x, void *d_y, void *stream);

/*
 * Expectation values of a generic operator (the measurements App. D takes with the
 * operator class): d_out[c] = sum_s x[s][c] (O x)[s][c] for each of the k real
 * columns (k in {1, 2, 4, 8}; <x|O|x> when O is symmetric), or, for complex vectors
 * (k = 1), d_out[0] + i d_out[1] = sum_s conj(x_s) (O x)_s.  The product is the one of
 * dcs_operator_apply, but no y is stored: each row's contribution is summed in FP64,
 * every workgroup writes its sum to d_ws, and a second kernel adds those in a fixed
 * order (strided per thread, then a fixed tree), so the result does not depend on timing.  d_out is device memory of k
 * doubles (2 for complex vectors); d_ws of at least the bytes
 * dcs_operator_expectation_workspace_size gives (caller-owned, reused freely between
 * calls, not shared by calls that overlap).  Errors as dcs_operator_apply, and
 * DCS_EINVAL for a NULL output or workspace or a workspace too small.  Asynchronous
 * on `stream`.
 */
int dcs_operator_expectation_workspace_size(const dcs_sector *sector, const dcs_operator *op, int k,
                                            size_t *bytes);
int dcs_operator_expectation(const dcs_sector *sector, const dcs_operator *op, int dtype, int k,
                             const void *d_x, double *d_out, void *d_ws, size_t ws_bytes, void *stream);

/* ========================================================================== */
/* Batched: many sectors in one launch                                        */
/* ========================================================================== */

/*
 * A plan applies H to one vector per sector for num_sectors sectors in a
 * single persistent launch.  Sector s uses terms[s] with couplings
 * d_jxy[s], d_jz[s] (device FP64 arrays; the pointers are recorded, the
 * values are read at apply time).  The sectors may differ in L, n, Q and
 * split.  Every sector is in the one launch, except sectors with a split view
 * (Q = 2, see "Split product") whose tables are in device memory, or all
 * sectors with a split view when DCS_PLAN_HYBRID=1 is set at creation: those
 * run their own product, in the form the autotuner keeps for them
 * (dcs_hamiltonian_apply): after the launch on the caller's stream at the
 * first apply of a dtype, later beside it on three streams of the plan
 * (created with it, default priority), forked from and joined back to the
 * caller's stream with events, so the call is still ordered on that stream.
 * Tiles go to the workgroups through per-XCD counters; every row is written
 * by one thread, so the result does not depend on the schedule.  The plan
 * does not own the sectors or terms; they must outlive it.
 */
int dcs_plan_create(int num_sectors, dcs_sector *const *sectors, dcs_terms *const *terms,
                    const double *const *d_jxy, const double *const *d_jz, dcs_plan **out);
int dcs_plan_destroy(dcs_plan *plan);

/* y_s = H_s x_s for every sector s; d_x[s], d_y[s] are device vectors of
 * D_s elements of dtype (k = 1).  Calls on one plan must not overlap in time
 * (they share its tile counters). */
int dcs_plan_apply(const dcs_plan *plan, int dtype, const void *const *d_x, void *const *d_y,
                   void *stream);

/* ========================================================================== */
/* Lanczos (Sec. 2.1 and App. D name it; the iteration is the textbook one)   */
/* ========================================================================== */

/*
 * Device workspace bytes for dcs_lanczos with these arguments.
 */
int dcs_lanczos_workspace_size(const dcs_sector *sector, int vec_dtype, int steps, int reorth,
                               int num_vec, size_t *bytes);

/*
 * Lanczos on the sector with FP64 scalars and vectors of vec_dtype:
 *   v_0 = v0/|v0|;  w = H v_j - beta_{j-1} v_{j-1};  alpha_j = v_j.w;
 *   w -= alpha_j v_j;  re-orthogonalise (reorth);  beta_j = |w|;  v_{j+1} = w/beta_j.
 * Dot products, norms and the re-orthogonalisation coefficients are
 * accumulated in FP64 on the device; vectors are stored in vec_dtype.
 * DCS_REORTH_FULL stores the basis and re-orthogonalises against all of it
 * (classical Gram-Schmidt twice).  DCS_REORTH_NONE and DCS_REORTH_LOCAL keep
 * two unnormalised vectors u_j (v_j = u_j/|u_j|) and take two passes over the
 * vectors per step after w = H u_j: the dots u_j.w, u_{j-1}.w, u_j.u_{j-1},
 * then u_{j+1} = w/|u_j| - A u_{j-1} - B u_j with its norm.  NONE uses the
 * three-term coefficients (A, B) = (beta_{j-1}/|u_{j-1}|, alpha_j/|u_j|); LOCAL
 * solves the 2x2 Gram system so that H v_j is projected out of
 * span(v_{j-1}, v_j) exactly for the stored operands (alpha_j is then the
 * coefficient of v_j).  In these two modes steps 2.. are replayed from two
 * captured HIP graphs (one per parity of j; the launches read j from the
 * workspace) on a private stream ordered after and before `stream`;
 * DCS_LANCZOS_GRAPH=0 in the environment launches every step eagerly (the
 * results are identical bit for bit).
 * Stops early when beta_j <= 1e-12 max_i(|alpha_i|, beta_i) or after D steps.
 * The Ritz values (eigenvalues of the tridiagonal T, Sturm bisection in FP64 on
 * the device) are returned in increasing order.
 *
 * d_v0: start vector (D elements, vec_dtype, device; not modified).
 * h_alpha[steps], h_beta[steps]: host outputs (beta has steps_done-1 valid entries).
 * h_steps_done: host output.  h_eig[num_eig]: the num_eig lowest Ritz values.
 * d_vecs: if not NULL, receives the normalised Ritz vectors of the num_vec
 * (>= 1) lowest Ritz values, vector e at d_vecs + e*D (vec_dtype; the lowest
 * num_vec states that App. D asks for).  Each is sum_j s_j v_j with s the
 * eigenvector of T for that Ritz value (inverse iteration in FP64 on the
 * device), assembled from the stored basis (DCS_REORTH_FULL) or by repeating
 * the recurrence once for all of them (other modes).  Only the first
 * min(num_vec, steps_done) are written.  Excited Ritz vectors converge later
 * than the ground vector; the caller picks `steps` for the states it wants.
 * num_vec must match the value given to dcs_lanczos_workspace_size.
 * Synchronises `stream` before returning (the outputs are on the host).
 */
int dcs_lanczos(const dcs_sector *sector, const dcs_terms *terms, const double *d_jxy,
                const double *d_jz, const double *d_h, int vec_dtype, int steps, int reorth,
                const void *d_v0, double *h_alpha, double *h_beta, int *h_steps_done,
                int num_eig, double *h_eig, void *d_vecs, int num_vec, void *d_workspace,
                size_t workspace_bytes, void *stream);

/*
 * dcs_lanczos for a generic operator (dcs_operator_create) in place of the XXZ
 * terms: the same iteration, re-orthogonalisation modes, Ritz values and vectors,
 * workspace (dcs_lanczos_workspace_size) and graph replay, with w = O v from
 * dcs_operator_apply's kernel.  O must be real symmetric on the sector (a real
 * operator whose terms sum to a symmetric matrix: Sec. 4.1's Hamiltonians built
 * from operator strings); the call does not check that.  Real vectors only
 * (DCS_F32 / DCS_F64); a complex operator is DCS_EINVAL.
 */
int dcs_lanczos_operator(const dcs_sector *sector, const dcs_operator *op, int vec_dtype,
                         int steps, int reorth, const void *d_v0, double *h_alpha,
                         double *h_beta, int *h_steps_done, int num_eig, double *h_eig,
                         void *d_vecs, int num_vec, void *d_workspace, size_t workspace_bytes,
                         void *stream);

/*
 * Eigenvalues of a symmetric tridiagonal matrix (diagonal h_alpha[m],
 * off-diagonal h_beta[m-1]) by Sturm-sequence bisection in FP64 on the
 * device; h_eig receives the num_eig lowest in increasing order.  Exposed so
 * the eigensolve step of dcs_lanczos can be checked on its own.
 */
int dcs_tridiag_eigvals(const double *h_alpha, const double *h_beta, int m, int num_eig,
                        double *h_eig, int device);

#ifdef __cplusplus
}
#endif

#endif /* DCS_H */
