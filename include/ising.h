/*
 * ising.h — C ABI of libising: exact degeneracy tables g(E, M) and partition
 * functions of finite Ising systems, computed on an AMD Instinct MI355X
 * (gfx950).
 *
 * The operation (Peretyatko et al., "Rigorous Calculation of the Partition
 * Function for the Finite Number of Ising Spins"):
 *   - Section 2, Eq. (1): H = -(1/2) sum_i sum_{j in nbr(i)} J_ij S_i S_j - h sum_i S_i.
 *     The factor 1/2 over the double neighbour sum counts each bond once, so
 *     for a bond multiset the exchange energy is E = -sum_b J_b s_i s_j and
 *     H = E - h M, with M = sum_i s_i the spin excess.
 *   - Section 2, the discussion after Eq. (2): every one of the 2^N
 *     configurations maps to a pair (E, M); the degeneracy multiplicity
 *     g(E, M) is the number of configurations with that pair.
 *   - Section 2, Eq. (2): Z_N(h, T) = sum over configurations of exp(-H/T)
 *     = sum_{E,M} g(E, M) exp(-(E - h M)/T), with k_B = 1.
 *   - Section 3 (a-d): the configurations are enumerated exhaustively as
 *     bit vectors and the work is split into independent ranges.
 *
 * Conventions used throughout:
 *   - spin u is "up" (s_u = +1) when its bit is set; n_up = number of up
 *     spins; M = 2 n_up - N.
 *   - the dense table g is uint64, row-major [n_e][n_m] with n_e = 2S + 1,
 *     n_m = N + 1, S = sum_b |J_b| over the bonds as given; entry
 *     g[(E - e_min) * n_m + n_up] with e_min = -S.
 *   - all functions are extern "C", never throw, and return ising_status
 *     (0 = success).  On failure ising_last_error() gives a message for the
 *     calling thread.
 *   - device pointers are addresses in the current HIP device's memory
 *     (e.g. torch.Tensor.data_ptr() of a CUDA tensor on ROCm); `stream` is a
 *     hipStream_t passed as void* (NULL = the default stream).  Calls that
 *     take a stream are asynchronous and stream-ordered: launch errors are
 *     returned at once, faults surface at the caller's next synchronisation.
 *   - the caller owns every buffer passed in; the library never frees or
 *     reallocates caller memory.
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ising_status {
  ISING_OK = 0,
  ISING_EINVAL = -1,            /* bad argument (null pointer, bad size, bad shape) */
  ISING_ETOO_MANY_SPINS = -2,   /* n_spins < 1 or > 64 */
  ISING_EBOND = -3,             /* bond endpoint out of range, or a self-bond i == j */
  ISING_ERANGE = -4,            /* couplings too large: S > 2^20, or histogram exceeds LDS */
  ISING_EHIP = -5,              /* a HIP runtime call failed (message has the HIP error) */
  ISING_ENOMEM = -6,            /* host or device allocation failed */
  ISING_EUNSUPPORTED = -7       /* valid input outside what the library handles
                                   (e.g. more than 8 distinct coupling values) */
} ising_status;

/* A finite Ising system: N spins and a multiset of bonds (i, j, J) with
 * integer couplings (Section 2, Eq. (1): the paper's J_ij may be sign-changing
 * and long-range).  Repeated pairs are allowed and add up.  All three arrays
 * are host pointers of length n_bonds; they are read during
 * ising_plan_create only and may be freed afterwards. */
typedef struct ising_lattice {
  int32_t n_spins;              /* 1 .. 64 */
  int32_t n_bonds;              /* >= 0 */
  const int32_t *bond_i;        /* endpoint sites, 0 .. n_spins-1 */
  const int32_t *bond_j;        /* endpoint sites, != bond_i */
  const int32_t *bond_J;        /* couplings, |J| <= 2^20 */
} ising_lattice;

/* Optional launch/decomposition choices; 0 in a field means "choose". */
typedef struct ising_tune {
  int32_t inner_bits;           /* k: configurations per chunk = 2^k (tile_bits .. 25) */
  int32_t tile_bits;            /* j: independent-set spins walked per block of 2^j steps (1 .. 8) */
  int32_t waves_per_block;      /* 1 .. 16 (64 lanes per wave) */
  int32_t replicas;             /* LDS histogram copies per block: 1, 2, 4, 8 or 16 */
  int32_t max_blocks;           /* grid cap */
  int32_t prefix_bits;          /* N - k: log2 of the chunk count, used when inner_bits is 0 */
} ising_tune;

/* Opaque, immutable after creation.  Safe to use from several threads and
 * streams at once with distinct outputs.  Device constants are uploaded on
 * the first launch on each device and owned by the plan. */
typedef struct ising_plan ising_plan;

/* Validate the lattice, merge repeated pairs, choose the spin ordering, the
 * chunk decomposition and the histogram geometry.  Host-only: makes no HIP
 * call.  `tune` may be NULL.  On success *plan receives a new plan that the
 * caller releases with ising_plan_destroy. */
ising_status ising_plan_create(const ising_lattice *lattice, const ising_tune *tune,
                               ising_plan **plan);

/* Release a plan and its device constants.  NULL is accepted.  The caller
 * must ensure no launch that uses the plan is still running. */
ising_status ising_plan_destroy(ising_plan *plan);

/* Dense table shape of the plan: *n_e = 2S + 1, *n_m = N + 1, *e_min = -S. */
ising_status ising_hist_shape(const ising_plan *plan, int32_t *n_e, int32_t *n_m,
                              int32_t *e_min);

/* Enumeration order (Section 3d: the configuration space is split into
 * independent ranges).  The plan renames spins to bit positions: site u is
 * bit bit_of_site[u] (array of n_spins entries, filled if non-NULL).  Chunk c
 * is the set of 2^inner_bits configurations whose bits inner_bits .. N-1 equal
 * c; there are *n_chunks = 2^(N - inner_bits) chunks.  Any of the outputs may
 * be NULL. */
ising_status ising_plan_layout(const ising_plan *plan, int32_t *bit_of_site,
                               int32_t *inner_bits, int32_t *tile_bits, uint64_t *n_chunks);

/* g(E, M) of all 2^N configurations into the device table g_dev
 * ([n_e][n_m] uint64, overwritten). */
ising_status ising_enumerate(const ising_plan *plan, uint64_t *g_dev, void *stream);

/* Add to g_dev the counts of the configurations in chunks
 * [first_chunk, first_chunk + n_chunks) (see ising_plan_layout).  Disjoint
 * ranges sum to the full table, which is how work is sharded or resumed.
 * Fails with ISING_EINVAL if the range exceeds the chunk count. */
ising_status ising_enumerate_range(const ising_plan *plan, uint64_t first_chunk,
                                   uint64_t n_chunks, uint64_t *g_dev, void *stream);

/* The same table as ising_enumerate, from half of the configurations: every
 * H of Eq. (1) at h = 0 is even in the spins, so a global spin flip maps
 * (E, M) to (E, -M) and g(E, M) = g(E, -M).  This enumerates the
 * configurations whose top plan bit (a prefix spin) is up, i.e. chunks
 * [n_chunks/2, n_chunks), then sets g(E, M) to the sum of their counts at M
 * and -M.  2^(N-1) configurations are enumerated for 2^N covered.  Plans with
 * a single chunk fall back to the full enumeration.  g_dev as in
 * ising_enumerate (overwritten). */
ising_status ising_enumerate_symmetric(const ising_plan *plan, uint64_t *g_dev, void *stream);

/* log Z(T, h) of Eq. (2) in FP64 from a dense table on the device:
 *   logz[a * nh + b] = log sum_{g>0} g(E,M) exp(-(E - h_b M)/T_a).
 * g_dev: [n_e][n_m] uint64 with n_m = n_spins + 1 and e_min its first energy.
 * T_dev[nT], h_dev[nh], logz_dev[nT * nh]: FP64 device arrays.  T must be
 * positive and finite; other T give NaN.  An all-zero table gives -inf. */
ising_status ising_logz(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                        int32_t n_spins, const double *T_dev, int32_t nT,
                        const double *h_dev, int32_t nh, double *logz_dev, void *stream);

/* Thermal moments under p(E, M) = g exp(-(E - hM)/T) / Z, each [nT][nh] FP64:
 *   mean_E = <E> (exchange energy), mean_M = <M>,
 *   heat_capacity = Var(E - h M) / T^2, susceptibility = Var(M) / T
 * (totals, not per spin; variances from centred sums).  Any output may be
 * NULL; logz_dev (optional) receives log Z as in ising_logz. */
ising_status ising_moments(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                           int32_t n_spins, const double *T_dev, int32_t nT,
                           const double *h_dev, int32_t nh, double *logz_dev,
                           double *mean_E, double *mean_M, double *heat_capacity,
                           double *susceptibility, void *stream);

/* ------------------------------------------------------------------------ */
/* Derivatives of log Z (for automatic differentiation).                    */
/* ------------------------------------------------------------------------ */

/* First and second derivatives of log Z(T, h) of Eq. (2), each [nT][nh] FP64
 * on the device (any output may be NULL), from differentiating the sum over
 * configurations with H = E - h M:
 *   d_T  = <H>/T^2,   d_h  = <M>/T,
 *   d_TT = Var(H)/T^4 - 2 <H>/T^3,
 *   d_Th = (Cov(H, M)/T - <M>)/T^2,   d_hh = Var(M)/T^2.
 * Inputs and error behaviour as ising_moments. */
ising_status ising_logz_derivatives(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                                    int32_t n_spins, const double *T_dev, int32_t nT,
                                    const double *h_dev, int32_t nh, double *logz_dev,
                                    double *d_T, double *d_h, double *d_TT, double *d_Th,
                                    double *d_hh, void *stream);

/* Per-configuration weights of a loss L = sum_{a,b} grad[a][b] log Z(T_a, h_b):
 * every configuration of bin (E, M) contributes
 *   W(E, M) = sum_{a,b} grad[a][b] exp(-(E - h_b M)/T_a - logz[a][b]) / T_a
 * (its Boltzmann probability at (T_a, h_b) times grad / T_a) to
 * dL/dJ_b = sum over configurations of W s_i s_j (Eq. (1): H depends on J_b
 * through -J_b s_i s_j).  g_dev, n_e, n_m, e_min, n_spins describe the
 * table as in ising_logz; logz_dev and grad_dev are [nT][nh] FP64 (logz as
 * returned by ising_logz for the same table and grid); W_dev receives the
 * dense [n_e][n_m] FP64 table (overwritten; 0 on empty bins). */
ising_status ising_bin_weights(const uint64_t *g_dev, int32_t n_e, int32_t n_m, int32_t e_min,
                               int32_t n_spins, const double *T_dev, int32_t nT,
                               const double *h_dev, int32_t nh, const double *logz_dev,
                               const double *grad_dev, double *W_dev, void *stream);

/* Bytes of device workspace ising_bond_backward needs for this plan (on the
 * current device).  Fails with ISING_EUNSUPPORTED when the backward cannot
 * run for this lattice (more than 512 distinct bond pairs, or a weight table
 * too large for the LDS); the message says which. */
ising_status ising_bond_workspace(const ising_plan *plan, size_t *bytes);

/* dJ[b] = sum over all 2^N configurations of W(E, M) s_i s_j for every input
 * bond b = (i, j) of the plan's lattice, in input order (repeated pairs get
 * the same value).  With W from ising_bin_weights this is dL/dJ_b.  The
 * enumeration is recomputed (nothing from the forward pass is stored); W is
 * summed in FP64 in a fixed order, so results are reproducible run to run.
 * W_dev: dense [n_e][n_m] FP64 table (ising_hist_shape of the plan); dJ_dev:
 * [n_bonds] FP64 (overwritten); workspace: device memory of at least
 * ising_bond_workspace bytes, used only during the call's stream order.  All
 * are device pointers. */
ising_status ising_bond_backward(const ising_plan *plan, const double *W_dev, double *dJ_dev,
                                 void *workspace, size_t workspace_bytes, void *stream);

/* The same dJ from half of the configurations.  A global spin flip keeps the
 * exchange energy E of Eq. (1) (it is even in the spins) and every product
 * s_i s_j, and negates M, so the sum over all configurations equals the sum
 * over those whose top spin (in the plan's order) is up, each weighted by
 * W(E, M) + W(E, -M); the paper's closing section suggests using such
 * symmetries.  About half the work; equal to ising_bond_backward up to FP64
 * summation order.  Lattices of at most tile_bits + 20 spins take the full
 * walk (their top spin is not among the spins every block walks in turn).
 * Arguments, workspace and errors as ising_bond_backward. */
ising_status ising_bond_backward_symmetric(const ising_plan *plan, const double *W_dev, double *dJ_dev,
                                           void *workspace, size_t workspace_bytes, void *stream);

/* The whole backward of log Z in one call: the gradient of a loss
 * L = sum_{a,b} G[a][b] log Z(T_a, h_b) (Eq. (2) for the plan's lattice) with
 * respect to the temperatures, the fields and the couplings, from the plan's
 * table g_dev (as ising_enumerate wrote it):
 *   grad_T[a] = sum_b G[a][b] <H>_ab / T_a^2,   grad_h[b] = sum_a G[a][b] <M>_ab / T_a
 *   (the averages in one pass over the bins with the given log Z as
 *   normaliser, <H> = sum p H / sum p, p = g exp(-(E - hM)/T - log Z); then
 *   contracted with G, each sum in index order),
 *   grad_J[k] = the ising_bond_backward sum of bond k with the weights of
 *   ising_bin_weights(G) (its halved form ising_bond_backward_symmetric when
 *   `symmetric` is nonzero); the weights are formed from the factorisation
 *   exp(-(E - hM)/T - log Z) = exp(-(E - E0)/T) exp((hM - E0)/T - log Z),
 *   E0 = -S the table's lowest energy, the sum over fields taken per (T, n_up)
 *   (each term summed directly where the split could leave the double range),
 *   so they equal ising_bin_weights' up to rounding.
 * T_dev[nT], h_dev[nh], logz_dev and G_dev [nT][nh] are FP64 device arrays
 * (logz as ising_logz returns it for the same table and grid).  Outputs are
 * FP64 device arrays of nT, nh and n_bonds entries; any may be NULL, and that
 * part is skipped (grad_J needs a plan the per-bond backward supports).
 * workspace: device memory of at least ising_logz_backward_workspace bytes,
 * used only in the call's stream order.  All kernels are issued on `stream`
 * in one call, with no host synchronisation. */
ising_status ising_logz_backward_workspace(const ising_plan *plan, int32_t nT, int32_t nh, size_t *bytes);
ising_status ising_logz_backward(const ising_plan *plan, const uint64_t *g_dev, const double *T_dev, int32_t nT,
                                 const double *h_dev, int32_t nh, const double *logz_dev, const double *G_dev,
                                 double *grad_T, double *grad_h, double *grad_J, int32_t symmetric,
                                 void *workspace, size_t workspace_bytes, void *stream);

/* ising_bond_backward without a workspace, for callers that cannot allocate
 * device memory at the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  It calls no allocating routine:
 * the per-block partial sums go to a static device array of the library
 * (4 MiB, at most 1024 blocks x 512 bond pairs; each device that runs it
 * holds its copy until the process ends), and the plan's device tables must
 * already be on the current device: one ising_bond_backward or
 * ising_bond_backward_symmetric call there uploads them, otherwise the call
 * fails with ISING_EINVAL.  Calls on one device share the array: calls that
 * overlap in time on one device race (serialise them on one stream).
 * W_dev, dJ_dev and the result are as in ising_bond_backward (the same
 * kernels in the same order, so the values are identical). */
ising_status ising_bond_backward_noalloc(const ising_plan *plan, const double *W_dev, double *dJ_dev,
                                         void *stream);

/* ------------------------------------------------------------------------ */
/* Batches: many lattices of uneven size in one persistent launch.          */
/* ------------------------------------------------------------------------ */

/* Opaque batch plan: one plan per lattice (same rules as ising_plan_create,
 * with one coupling-class count shared by all members so a single kernel
 * serves the batch; each member keeps its own tile width, chunk width and LDS
 * layout) and a work list of (lattice, task) units ordered largest lattice
 * first.  Immutable after creation, except for the
 * device work counter: launches that use the same batch plan must not
 * overlap in time (serialise them on one stream). */
typedef struct ising_batch_plan ising_batch_plan;

/* n lattices, 1 <= n <= 65535 (host array of n descriptors, read during the
 * call only); tune may be NULL.  Each member's chunk width is
 * tune.inner_bits (default 14, at most the member's N) unless
 * tune.prefix_bits is given, except that the smallest members, together
 * about one round of work units over 256 CUs (last in the work list), take
 * chunks of at most 2^12 configurations so the launch ends on short units;
 * tile_bits is an upper bound on each member's tile width; replicas,
 * waves_per_block and max_blocks apply to every member. */
ising_status ising_batch_plan_create(const ising_lattice *lattices, int32_t n, const ising_tune *tune,
                                     ising_batch_plan **plan);
ising_status ising_batch_plan_destroy(ising_batch_plan *plan);

/* Layout of the concatenated tables g_all: member i's dense [n_e[i]][n_m[i]]
 * uint64 table starts at element offsets[i]; offsets has n + 1 entries, the
 * last one being the total element count.  e_min[i] = -S_i.  Any output may
 * be NULL; arrays are caller-owned host memory. */
ising_status ising_batch_layout(const ising_batch_plan *plan, int64_t *offsets, int32_t *n_e, int32_t *n_m,
                                int32_t *e_min, int32_t *n_spins);

/* g(E, M) of every member into g_all (device, offsets[n] uint64,
 * overwritten), in one persistent launch. */
ising_status ising_batch_enumerate(const ising_batch_plan *plan, uint64_t *g_all_dev, void *stream);

/* The same tables from half of the configurations (the batched form of
 * ising_enumerate_symmetric): every member with at least two chunks is
 * enumerated over the chunks with its top spin up, then mirrored,
 * g(E, M) = h(E, M) + h(E, -M) (a global spin flip keeps E and negates M).
 * Bit-identical to ising_batch_enumerate.  Arguments as there. */
ising_status ising_batch_enumerate_symmetric(const ising_batch_plan *plan, uint64_t *g_all_dev, void *stream);

/* log Z and moments of every member on one (T, h) grid, as ising_moments;
 * each output (any may be NULL) is [n][nT][nh] FP64 on the device. */
ising_status ising_batch_moments(const ising_batch_plan *plan, const uint64_t *g_all_dev, const double *T_dev,
                                 int32_t nT, const double *h_dev, int32_t nh, double *logz_dev,
                                 double *mean_E, double *mean_M, double *heat_capacity,
                                 double *susceptibility, void *stream);

/* A captured HIP graph of {zero g_all, batched enumeration, batched
 * moments} with the given buffers baked in (nT or nh = 0 leaves the moments
 * out).  Replays reproduce ising_batch_enumerate + ising_batch_moments. */
typedef struct ising_graph ising_graph;
ising_status ising_batch_graph_create(const ising_batch_plan *plan, uint64_t *g_all_dev, const double *T_dev,
                                      int32_t nT, const double *h_dev, int32_t nh, double *logz_dev,
                                      double *mean_E, double *mean_M, double *heat_capacity,
                                      double *susceptibility, ising_graph **graph);
/* The same graph with the halved enumeration (ising_batch_enumerate_symmetric). */
ising_status ising_batch_graph_create_symmetric(const ising_batch_plan *plan, uint64_t *g_all_dev,
                                                const double *T_dev, int32_t nT, const double *h_dev, int32_t nh,
                                                double *logz_dev, double *mean_E, double *mean_M,
                                                double *heat_capacity, double *susceptibility, ising_graph **graph);
ising_status ising_graph_launch(const ising_graph *graph, void *stream);
ising_status ising_graph_destroy(ising_graph *graph);

/* Static text for a status code. */
const char *ising_status_str(ising_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *ising_last_error(void);

/* Library version string. */
const char *ising_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
