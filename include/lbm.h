/*
 * lbm.h -- C ABI of the list-based D3Q19 TRT lattice Boltzmann library for
 * AMD Instinct MI355X (gfx950).
 *
 * The method is that of Wittmann, Zeiser, Hager, Wellein, "Domain
 * decomposition and locality optimization for large-scale lattice Boltzmann
 * simulations": a sparse representation that stores only fluid cells in a
 * 1-D list together with an adjacency list (Sec. 2), assembled from a full
 * flag field through a numbering scheme and a contiguous index (Sec. 3), and
 * a D3Q19 two-relaxation-time pull sweep over that list (Sec. 1, Sec. 7).
 *
 * General conventions
 *  - Every pointer is a DEVICE pointer unless marked (host).
 *  - The caller owns all memory.  The library never allocates device memory;
 *    calls that need scratch space take a caller-provided workspace whose
 *    size is obtained by calling with workspace == NULL (size query).
 *  - The library keeps no global state, with one exception: the fixed
 *    per-device scratch array of lbm_moments_noalloc (see there).
 *  - Every call is ordered on `stream` (a hipStream_t, NULL = the null
 *    stream) and asynchronous, except the outputs marked "synchronous" which
 *    are returned to the host.
 *  - Every call returns an lbm_status and never aborts or throws.  Argument
 *    errors are detected on the host before any launch.  A launch failure
 *    reported by the HIP runtime returns LBM_EHIP; faults that surface later
 *    are reported by the caller's next synchronisation.
 *  - Indices: fluid cells are numbered 0..N_f-1 in key order ("contiguous
 *    index" I_c of Sec. 3, 0-based; solid cells get -1 where the paper writes
 *    0).  A box cell (x,y,z) of an nx*ny*nz box has linear index
 *    lin = x + nx*(y + ny*z).
 *  - PDF arrays are structure-of-arrays [19][stride] (Sec. 7): population i of
 *    list cell m lives at element i*stride + m.  Several geometries may share
 *    one set of arrays, each occupying columns [base, base + N_f) ("batched").
 *
 * D3Q19 numbering: i = 0 rest; 1,2 = +-x; 3,4 = +-y; 5,6 = +-z;
 * 7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0) 11 (1,0,1) 12 (-1,0,-1)
 * 13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1).
 * Opposite pairs are (2k-1, 2k).  Weights 1/3, 1/18 (axis), 1/36 (diagonal).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* bad argument: NULL required pointer, bad dims/enum, stride < n ... */
    LBM_ECAPACITY = -2,  /* output capacity too small; required size is returned */
    LBM_EOVERFLOW = -3,  /* index does not fit: 19*stride >= 2^32 or box >= 2^31 cells */
    LBM_EWORKSPACE = -4, /* workspace missing or smaller than the size query returned */
    LBM_EHIP = -5,       /* the HIP runtime reported an error */
    LBM_EBARRIER = -6,   /* persistent launch: a grid barrier exceeded its spin limit */
    LBM_ENONFINITE = -7  /* lbm_moments with LBM_FLAG_CHECK_FINITE: a total is NaN or infinite */
} lbm_status;

/* Numbering schemes (Sec. 3 "Numbering scheme"; Sec. 7 blocking factor and
 * Z-curve variants). */
typedef enum {
    LBM_ORDER_LEX = 0,     /* key = lin (x fastest) */
    LBM_ORDER_BLOCKED = 1, /* cubic blocks of edge b = order_param, blocks and the
                              cells inside a block both lexicographic; edge blocks
                              truncated; b = 1 is plain lexicographic */
    LBM_ORDER_MORTON1 = 2, /* Z curve, 1-bit interleave: bit k of x,y,z -> bit 3k,3k+1,3k+2 */
    LBM_ORDER_MORTON2 = 3, /* Z curve, 2-bit groups: bits [2k,2k+2) of x,y,z -> [6k,6k+2),
                              [6k+2,6k+4), [6k+4,6k+6) */
    LBM_ORDER_RANDOM = 4,  /* key = 4-round Feistel bijection of lin on [0, 4^h),
                              4^h >= box (smallest h >= 1); round r maps (L,R) ->
                              (R, L ^ (splitmix64(seed ^ (r << 32) ^ R) & (2^h - 1)));
                              seed = order_param.  A control ordering: the paper
                              allows any injective index function. */
    LBM_ORDER_HILBERT = 5  /* Hilbert curve on the enclosing 2^B cube (Sec. 3 names it):
                              Skilling's transposed index (AIP Conf. Proc. 707, 2004)
                              of (x, y, z), read level by level with x's bit the most
                              significant of each 3-bit digit */
} lbm_order;

/* PDF storage (the paper stores double precision, Sec. 7).  "Shifted" arrays
 * hold f_i - w_i.  F64 forms compute in FP64; F32/F16 forms compute in FP32.
 * Reductions (moments totals) are always accumulated in FP64.
 * LBM_F16_SHIFTED_SCALED stores 2^12 (f_i - w_i) in FP16: the same bytes as
 * LBM_F16_SHIFTED, but deviations down to 2^-26 stay in FP16's normal range
 * (shifted FP16 turns those below 2^-14 subnormal, which is what limits its
 * accuracy at small forcing); |f_i - w_i| must stay below 16 (a lattice
 * Boltzmann state has 0 <= f_i <= 1).  Multiplying by 2^12 and by 2^-12 is
 * exact, so the only rounding is the FP16 store, as in the unscaled form. */
typedef enum {
    LBM_F64 = 0,
    LBM_F64_SHIFTED = 1,
    LBM_F32 = 2,
    LBM_F32_SHIFTED = 3,
    LBM_F16_SHIFTED = 4,
    LBM_F16_SHIFTED_SCALED = 5
} lbm_storage;

enum {
    LBM_FLAG_NONTEMPORAL = 1, /* write the new PDFs with nontemporal stores (Sec. 7) */
    LBM_FLAG_CHECK_FINITE = 2, /* lbm_moments: read the totals back (synchronising the
                                  stream) and return LBM_ENONFINITE if one is NaN or
                                  infinite (a diverged run); ignored by the sweeps */
    /* Workgroup-to-XCD mapping of the sweep, bits [8, 16) of flags, a power of
     * two k: the hardware hands workgroup w to XCD w % 8; the sweep relabels
     * workgroups so that each XCD takes k consecutive list tiles before the
     * next XCD's k.  k = 1 keeps the hardware round robin; 0 (default) gives
     * each XCD one contiguous eighth of the list.  Results do not depend on it. */
    LBM_FLAG_XCD_CHUNK_SHIFT = 8,
    LBM_FLAG_XCD_CHUNK_MASK = 0xff00
};

typedef struct {
    int32_t nx, ny, nz;
    uint32_t periodic;    /* bit0 x, bit1 y, bit2 z; non-periodic out-of-box = solid */
    int32_t order;        /* lbm_order */
    uint32_t order_param; /* blocking factor b (BLOCKED) or seed (RANDOM) */
} lbm_geom;

/* TRT parameters.  tau_minus = 1/2 + magic / (tau_plus - 1/2); s+- = 1/tau+-.
 * force = body force G per unit volume (lattice units). */
typedef struct {
    double tau_plus;
    double magic;
    double force[3];
    int32_t storage; /* lbm_storage */
    int32_t flags;   /* LBM_FLAG_* */
} lbm_params;

/* One geometry of a batch: list columns [base, base + n), run with parameter
 * set params[param_index] of the call.  Segments are listed in increasing
 * order and do not overlap.  When any segment of a call names a set other than
 * 0, every non-empty segment must start on a multiple of 256 (a sweep tile),
 * so that no tile holds cells of two segments. */
typedef struct {
    int64_t base;
    int64_t n;
    int32_t param_index;
    int32_t pad;
} lbm_segment;

/*
 * lbm_build_adjacency -- assembly of the sparse representation (Sec. 3).
 *
 * Numbering scheme -> contiguous index -> adjacency.  Every box cell gets the
 * key of g->order; fluid cells are ranked by key (I_c, Sec. 3 "Contiguous
 * index generation": the rank the paper's octree merge of incell runs
 * computes, here an exclusive prefix count of fluid flags in key order); the
 * adjacency is found by inspecting each fluid cell's neighbourhood in the full
 * representation (Sec. 3, last paragraph of the assembly) with bounce-back
 * encoded implicitly (Sec. 2).  The result is independent of any launch
 * parameter (Sec. 8: the same geometry and numbering always produce exactly
 * the same sparse representation).
 *
 *  g         (host) box dims, periodicity, ordering.
 *  flag      uint8 [nz][ny][nx], nonzero = fluid.
 *  base      first list column of this geometry in the shared arrays.
 *  stride    row stride of adj (and of the PDF arrays); stride >= base + N_f.
 *  index_of  int32 [nx*ny*nz] or NULL: I_c of each box cell, -1 for solid.
 *  cell_of   int32 [cap] or NULL: lin of list cell m (cell_of[m], m < N_f).
 *            NULL = count-only pass: only *n_fluid is produced.
 *  adj       uint32 [18][stride] or NULL (compaction only).  Row k is
 *            direction i = k+1; entry adj[k*stride + base + m] =
 *              i*stride + base + I_c(x_m - c_i)   if that upstream cell (wrapped
 *                                                  in periodic directions) is fluid,
 *              opp(i)*stride + base + m           otherwise (bounce-back).
 *            The rest population is implicit (slot base + m of row 0).
 *  cap       capacity of cell_of in cells.
 *  n_fluid   (host, synchronous) N_f.  Set also when LBM_ECAPACITY is returned.
 *  workspace device scratch of *ws_bytes bytes; NULL = size query: *ws_bytes
 *            is set and nothing else happens.
 *  ws_bytes  (host, in/out) workspace size.
 * Errors: LBM_EINVAL (NULL g/flag/n_fluid/ws_bytes, dims <= 0, bad order,
 * b == 0, stride < base + N_f when adj given), LBM_EOVERFLOW (box >= 2^31 cells,
 * 19*stride >= 2^32), LBM_ECAPACITY (N_f > cap; nothing written), LBM_EWORKSPACE.
 */
lbm_status lbm_build_adjacency(const lbm_geom* g, const uint8_t* flag, int64_t base,
                               int64_t stride, int32_t* index_of, int32_t* cell_of,
                               uint32_t* adj, int64_t cap, int64_t* n_fluid, void* workspace,
                               size_t* ws_bytes, void* stream);

/*
 * lbm_init -- equilibrium initial state (the configurations start from rest:
 * rho = 1, u = 0; the TRT equilibrium is that of the sweep below, and the
 * paper's FLUP count (Sec. 7) starts from such a state).
 *
 * Writes f_i = w_i [rho0 + 3 c_i.u0 + 9/2 (c_i.u0)^2 - 3/2 |u0|^2] (minus w_i in
 * shifted storage, computed as w_i [(rho0 - 1) + ...]) for list cells [0, n)
 * of every row.  The element type of f follows p->storage.  To initialise a
 * batch member, offset f by its base (in elements).
 *  p      (host) parameters (only the storage is used; the other fields are
 *         checked by the sweeps that use them).
 *  n, stride  cells written and row stride of f ([19][stride]).
 *  f      PDF array, written (caller-owned).
 *  rho0   density; u0 (host) 3 doubles, or NULL for u0 = 0.
 * Errors: LBM_EINVAL (NULL p/f, n < 0, stride < n, bad storage, non-finite
 * rho0 or u0), LBM_EOVERFLOW (19*stride >= 2^32), LBM_EHIP.
 */
lbm_status lbm_init(const lbm_params* p, int64_t n, int64_t stride, void* f, double rho0,
                    const double* u0, void* stream);

/*
 * lbm_step -- n_steps D3Q19 TRT pull sweeps over list cells [0, n)
 * (Sec. 1, Sec. 2, Sec. 7: TRT on D3Q19, structure of arrays, pull scheme,
 * indirect addressing, optionally nontemporal stores; a batch of geometries
 * in one list is the paper's list of fluid cells holding several domains).
 *
 * Per cell m: gather g_0 = f[m], g_i = f[adj[i-1][m]]; rho = sum g;
 * j = sum c_i g_i; e+_i = w_i (rho + 9/2 (c_i.j)^2 - 3/2 |j|^2); e-_i = 3 w_i c_i.j;
 * f*_i = g_i - s+ ((g_i + g_opp)/2 - e+_i) - s- ((g_i - g_opp)/2 - e-_i) + 3 w_i c_i.G;
 * with a solid fraction ns (partial bounce-back): out_i = (1 - ns) f*_i + ns g_opp;
 * store out_i at element i*stride + m of the destination array.  In shifted
 * storage the same map acts on f - w with rho read as the density deviation.
 *
 *  p, n_params  (host) 1 <= n_params <= 65536 parameter sets.  All sets share
 *               one storage type and one set of launch flags (those of p[0]).
 *  seg, n_seg   (host) batch layout, or NULL/0 for one geometry [0, n).  Segments
 *               lie inside [0, n), in increasing order, without overlap
 *               (adjacency entries already carry each member's base).  Segment k
 *               runs with p[seg[k].param_index]; cells outside every segment
 *               with p[0].
 *  adj          uint32 [18][stride] from lbm_build_adjacency.
 *  ns           double [stride] solid fraction per list cell, or NULL (plain TRT).
 *  f_a, f_b     two PDF arrays [19][stride] of the storage type.  Step k reads the
 *               array written by step k-1 (f_a first): the result is in f_b if
 *               n_steps is odd, in f_a if even.
 *  persistent   0: one kernel launch per step.  1: a single cooperative launch
 *               runs all n_steps with a grid-wide barrier between steps (one
 *               workgroup per CU) and synchronises the stream to report
 *               LBM_EBARRIER.
 *  workspace, ws_bytes  device scratch for the persistent launch (a barrier
 *               block) and for per-segment parameter sets (a table of the sets
 *               and one int32 per 256-cell tile).  A call that needs it and gets
 *               workspace == NULL stores the size in *ws_bytes and does nothing
 *               else (size query); a call with one parameter set and
 *               persistent == 0 needs none (workspace may be NULL).
 * Every member's state is bitwise what a run of that member alone (same
 * parameters) gives, in either launch form.
 * Errors: LBM_EINVAL (NULL p/adj/f_a/f_b, f_a == f_b, n < 0, stride < n,
 * n_params outside [1, 65536], sets differing in storage or flags, bad storage, tau_plus <= 1/2,
 * non-finite parameters, bad segments: out of order, overlapping, outside
 * [0, n), param_index outside [0, n_params), a segment not starting on a tile
 * while sets differ), LBM_EOVERFLOW (19*stride >= 2^32), LBM_EWORKSPACE,
 * LBM_EHIP, LBM_EBARRIER (persistent only; synchronous check after the launch).
 */
lbm_status lbm_step(const lbm_params* p, int32_t n_params, const lbm_segment* seg, int32_t n_seg,
                    int64_t n, int64_t stride, const uint32_t* adj, const double* ns,
                    void* f_a, void* f_b, int32_t n_steps, int32_t persistent,
                    void* workspace, size_t* ws_bytes, void* stream);

/*
 * lbm_step_batch -- lbm_step (same arguments, same results bit for bit) that
 * reads the adjacency codes of lbm_compress_adjacency / lbm_narrow_codes
 * instead of adj where a tile allows it, in either launch form: the byte
 * reduction of lbm_step_c8 for a batch of geometries with per-segment
 * parameter sets, and in the single persistent launch.
 *
 *  codes8   int8 [18][stride] from lbm_narrow_codes, or NULL (no 8-bit codes).
 *  codes, tile_records  from lbm_compress_adjacency for the same n, stride and
 *           adj, or both NULL (full list; codes8 must then be NULL too).
 *  The other arguments as lbm_step.
 * With persistent = 0 the call only enqueues kernel launches on `stream` (no
 * allocation, memset, copy or synchronisation), so a caller may capture it in
 * a HIP graph with the workspace allocated beforehand: one graph launch then
 * runs all n_steps sweeps, each with the hardware's workgroup dispatch, and
 * gives the per-step launches' results bit for bit.  The persistent launch
 * synchronises the stream to report LBM_EBARRIER and cannot be captured.
 * Errors: as lbm_step, and LBM_EINVAL for codes8 without codes or only one of
 * codes and tile_records.
 */
lbm_status lbm_step_batch(const lbm_params* p, int32_t n_params, const lbm_segment* seg,
                          int32_t n_seg, int64_t n, int64_t stride, const int8_t* codes8,
                          const int16_t* codes, const int32_t* tile_records, const uint32_t* adj,
                          const double* ns, void* f_a, void* f_b, int32_t n_steps,
                          int32_t persistent, void* workspace, size_t* ws_bytes, void* stream);

/*
 * lbm_step_adjoint -- transposed Jacobian of one lbm_step (FP64 storage only):
 * the reverse-mode derivative of the sweep of Sec. 7 that gives the gradient
 * of the permeability (mean flux, proportional to the mean x velocity) with
 * respect to a per-cell partial-bounce-back solid fraction.  The paper has no
 * adjoint; the step is the exact transpose of the forward map written above
 * (derived by hand from it), applied in reverse over checkpointed states.
 *
 * Forward: f^{t+1} = step(f^t; ns).  Given lam_next = lambda^{t+1} it writes
 * lambda^t = (d f^{t+1} / d f^t)^T lambda^{t+1} -- the local transposed
 * collision Jacobian applied per cell and scattered back through the same
 * adjacency (every slot of lam_t is written exactly once: the pull is a
 * permutation) -- and accumulates grad_ns[m] += sum_i lambda^{t+1}_i(m)
 * (g_opp(i) - f*_i), the derivative through the solid fraction.
 * With lam_next == NULL it writes the seed lambda^T = dJ/df^T of the
 * objective J = (1/n) sum_m (j_x(m) + G_x/2) (mean x velocity of the state
 * after the last step, i.e. the mean flux that sets the permeability; the
 * value lbm_objective returns); then grad_ns is not touched.
 *
 *  p        (host) parameters of the forward step (storage F64 or F64_SHIFTED).
 *  n, stride, adj  as lbm_step.
 *  f_t      state entering step t ([19][stride], F64 or F64_SHIFTED).
 *  ns       solid fraction [stride] or NULL (then grad_ns is ignored).
 *  lam_next double [19][stride] or NULL; lam_t double [19][stride] (output).
 *  grad_ns  double [stride], accumulated (+=); caller zeroes it.
 *  p->flags the sweep's launch options apply (nontemporal stores of lam_t,
 *           workgroup-to-XCD mapping); results do not depend on them.
 * Errors: LBM_EINVAL (NULL p/adj/f_t/lam_t, n <= 0, stride < n, storage not
 * FP64), LBM_EOVERFLOW, LBM_EHIP.
 */
lbm_status lbm_step_adjoint(const lbm_params* p, int64_t n, int64_t stride, const uint32_t* adj,
                            const void* f_t, const double* ns, const double* lam_next,
                            double* lam_t, double* grad_ns, void* stream);

/*
 * lbm_step_adjoint_c16 -- lbm_step_adjoint (lam_next != NULL) with the slots
 * rebuilt from the 16-bit codes of lbm_compress_adjacency instead of read
 * from adj (552 - 36 bytes per cell-step); tiles with escape codes read adj.
 * Results are bitwise those of lbm_step_adjoint.
 *
 *  codes, tile_records  from lbm_compress_adjacency for the same n, stride
 *        and adj.  The other arguments as lbm_step_adjoint; the seed
 *        (lam_next == NULL) is not offered here.
 * Errors: LBM_EINVAL (NULL p/codes/tile_records/adj/f_t/lam_next/lam_t,
 * n <= 0, stride < n, storage not FP64), LBM_EOVERFLOW, LBM_EHIP.
 */
lbm_status lbm_step_adjoint_c16(const lbm_params* p, int64_t n, int64_t stride,
                                const int16_t* codes, const int32_t* tile_records,
                                const uint32_t* adj, const void* f_t, const double* ns,
                                const double* lam_next, double* lam_t, double* grad_ns,
                                void* stream);

/*
 * lbm_step_adjoint_c8 -- lbm_step_adjoint_c16 reading the 8-bit codes of
 * lbm_narrow_codes in narrow tiles (552 - 54 bytes per cell-step there), the
 * 16-bit codes in the other escape-free tiles and adj in tiles with escapes.
 * Results are bitwise those of lbm_step_adjoint (every form rebuilds the same
 * slots).
 *
 *  codes8  int8 [18][stride] from lbm_narrow_codes for the same codes and
 *        tile_records (which carry the narrow flags).  The other arguments as
 *        lbm_step_adjoint_c16.
 * Errors: as lbm_step_adjoint_c16, and LBM_EINVAL for NULL codes8.
 */
lbm_status lbm_step_adjoint_c8(const lbm_params* p, int64_t n, int64_t stride,
                               const int8_t* codes8, const int16_t* codes,
                               const int32_t* tile_records, const uint32_t* adj,
                               const void* f_t, const double* ns, const double* lam_next,
                               double* lam_t, double* grad_ns, void* stream);

/*
 * lbm_moments -- macroscopic fields and FP64 totals of a stored state (the
 * density and velocity of each fluid cell, from the populations the next pull
 * sweep of Sec. 7 gathers; the totals are what the mass-conservation and
 * flux checks and the precision comparison read).
 *
 * Per list cell, from the populations it gathers through adj (the values the
 * next sweep would read): rho = sum g (1 + sum h in shifted storage),
 * u = j + G/2 with the force G of the cell's segment.  Totals per segment:
 * {sum rho, sum u_x, sum u_y, sum u_z}, accumulated in FP64 double-double in a
 * fixed order, so results do not depend on timing.
 *
 *  p, n_params  (host) parameter sets as in lbm_step (the force and storage
 *        are used); segment k reads p[seg[k].param_index].
 *  n, stride, adj, f  the state (layout of lbm_step, storage p[0].storage).
 *  rho   double [n] or NULL.   u  double [3][n] (rows x, y, z) or NULL.  Only
 *        the cells of the segments are written.
 *  seg, n_seg  (host) segments, or NULL/0 for one segment [0, n).
 *  totals double [4 * max(n_seg,1)] or NULL.
 *  workspace, ws_bytes  scratch for the reduction (query with workspace NULL);
 *        not needed when totals == NULL.
 *  With LBM_FLAG_CHECK_FINITE in p[0].flags and totals given, the call waits
 *  for the totals and returns LBM_ENONFINITE if any of them is NaN or
 *  infinite (the fields are written either way).
 * Errors: LBM_EINVAL, LBM_EOVERFLOW, LBM_EWORKSPACE, LBM_EHIP, LBM_ENONFINITE.
 */
lbm_status lbm_moments(const lbm_params* p, int32_t n_params, int64_t n, int64_t stride,
                       const uint32_t* adj, const void* f, double* rho, double* u,
                       const lbm_segment* seg, int32_t n_seg, double* totals, void* workspace,
                       size_t* ws_bytes, void* stream);

/*
 * lbm_objective -- the objective the adjoint differentiates: per segment the
 * mean x velocity J = (1/N) sum_m (j_x(m) + G_x/2) over its N cells, the mean
 * flux that sets the permeability k = nu J / G_x (nu = (tau+ - 1/2)/3).  The
 * sum is lbm_moments' FP64 double-double total, divided by N on the device,
 * so J equals totals[1] / N of lbm_moments bit for bit.
 *
 *  p, n_params, n, stride, adj, f, seg, n_seg  as lbm_moments.
 *  J     double [max(n_seg, 1)] (output; an empty segment gives NaN).
 *  workspace, ws_bytes  as lbm_moments with totals (query with workspace NULL).
 * Errors: LBM_EINVAL, LBM_EOVERFLOW, LBM_EWORKSPACE, LBM_EHIP.
 */
lbm_status lbm_objective(const lbm_params* p, int32_t n_params, int64_t n, int64_t stride,
                         const uint32_t* adj, const void* f, const lbm_segment* seg,
                         int32_t n_seg, double* J, void* workspace, size_t* ws_bytes,
                         void* stream);

/*
 * lbm_moments_noalloc -- lbm_moments without a workspace, for callers that
 * cannot allocate device memory: code under stream capture, tight serving
 * loops, harnesses that forbid allocation.  The caller still passes the
 * state and the outputs.
 *
 * Same arguments as lbm_moments minus workspace / ws_bytes.  rho and u are
 * bitwise those of lbm_moments; each total is the same double-double sum taken
 * in another grouping (a workgroup covers several tiles), so it agrees with
 * lbm_moments' to about 1e-30 relative before the final rounding.  The partial
 * sums live in a fixed array of the library, 4096 partials (256 KiB) per GPU,
 * held until the process ends; the first call on a device looks up its
 * address (no allocation).  No input size exceeds it: the cells per workgroup
 * grow with the segment.  Every call on one GPU shares that array, so calls
 * that overlap on one GPU (other streams, other threads) race: order them.
 * Errors: LBM_EINVAL, LBM_EOVERFLOW, LBM_EHIP, LBM_ENONFINITE (with
 * LBM_FLAG_CHECK_FINITE, as lbm_moments).
 */
lbm_status lbm_moments_noalloc(const lbm_params* p, int32_t n_params, int64_t n, int64_t stride,
                               const uint32_t* adj, const void* f, double* rho, double* u,
                               const lbm_segment* seg, int32_t n_seg, double* totals,
                               void* stream);

/*
 * lbm_check_adjacency -- checked mode of an adjacency list (a validation and
 * debugging aid for adjacencies built or loaded outside the library).
 *
 * For the n list cells of one geometry at columns [base, base + n), with
 * the entry contract of lbm_build_adjacency (Sec. 2: the adjacency list;
 * Sec. 7: the pull scheme): every entry must lie in rows 1..18 of those
 * columns (in particular below 19 * stride), and the 18 n entries must be a
 * permutation of those 18 n slots, each referenced exactly once -- the
 * property that makes the pull sweep read every population once and the
 * adjoint and in-place scatters write every slot once.  The check never uses
 * an out-of-range entry as an address.
 *  base, n, stride, adj  the geometry's columns and the [18][stride] list.
 *  result  (host, synchronous) int64 [2]: [0] entries out of range, [1] slots
 *          of the 18 n not referenced exactly once (0 and 0: valid).
 *  workspace, ws_bytes  scratch of 18 n + 64 uint32 (query with workspace
 *          NULL).
 * Errors: LBM_EINVAL (base < 0, n < 0, NULL ws_bytes / adj / result),
 * LBM_EOVERFLOW (19*stride >= 2^32), LBM_EWORKSPACE, LBM_EHIP.  A list that
 * fails the check is reported through result with LBM_OK.
 */
lbm_status lbm_check_adjacency(int64_t base, int64_t n, int64_t stride, const uint32_t* adj,
                               int64_t* result, void* workspace, size_t* ws_bytes,
                               void* stream);

/*
 * lbm_partition_stats -- communication metrics of cutting the list into
 * n_chunks near-equal chunks (Sec. 2: a solver on N processes cuts the 1-D
 * list into N equal chunks, some smaller by one cell; Sec. 7 and Fig. 7:
 * number of neighbour partitions and of remote links per partition).
 *
 * Chunk k holds list cells [floor(k n / G), floor((k+1) n / G)), G = n_chunks.
 * A remote link is an adjacency entry of a cell in chunk a that streams
 * (not bounce-back) from a cell of another chunk b: the PDF chunk a would
 * have to receive each step.  Per chunk it reports:
 *  remote_links    int64 [G]: number of remote links;
 *  neighbours      int32 [G]: number of distinct chunks it pulls from (the
 *                  relation is symmetric for a pull adjacency);
 *  interface_cells int32 [G]: cells with at least one remote link.
 *  workspace, ws_bytes: scratch (query with workspace == NULL).
 * Errors: LBM_EINVAL (n_chunks <= 0 or > 16384, n <= 0, NULL outputs),
 * LBM_EOVERFLOW, LBM_EWORKSPACE, LBM_EHIP.
 */
lbm_status lbm_partition_stats(int64_t n, int64_t stride, const uint32_t* adj, int64_t n_chunks,
                               int64_t* remote_links, int32_t* neighbours,
                               int32_t* interface_cells, void* workspace, size_t* ws_bytes,
                               void* stream);

/*
 * lbm_compress_adjacency -- 16-bit re-encoding of the adjacency list
 * (byte reduction of the sweep over the sparse representation of Sec. 2,
 * whose adjacency list is read by every pull update of Sec. 7: in FP64 it
 * is 72 of the 376 bytes an update moves).
 *
 * List tiles are 256 consecutive cells.  Per tile t and direction i = k + 1
 * an int32 offset o = tile_records[t * 20 + k] is chosen, and entry
 * adj[k][m] = i * stride + src becomes the int16
 *   codes[k * stride + m] = src - m - o
 * when that lies in [-32766, 32767]; an implicit bounce-back entry
 * (opp(i) * stride + m) becomes -32768, any other entry -32767 ("escape").
 * tile_records[t * 20 + 18] = number of escapes in tile t, [t * 20 + 19] = 0.
 * The encoding is lossless.
 *
 *  adj           uint32 [18][stride] from lbm_build_adjacency (input).
 *  codes         int16  [18][stride] (output; columns >= n untouched).
 *  tile_records  int32  [ceil(n / 256) * 20] (output).
 *  n_escapes     (host) number of escape codes written.
 *  workspace, ws_bytes  2056 bytes of device scratch for partial sums
 *        (query with workspace NULL).  The call synchronizes the stream to
 *        return n_escapes.
 * Errors: LBM_EINVAL (NULL pointers, n <= 0), LBM_EOVERFLOW, LBM_EWORKSPACE,
 * LBM_EHIP.
 */
lbm_status lbm_compress_adjacency(int64_t n, int64_t stride, const uint32_t* adj, int16_t* codes,
                                  int32_t* tile_records, int64_t* n_escapes, void* workspace,
                                  size_t* ws_bytes, void* stream);

/*
 * lbm_step_c16 -- n_steps TRT pull sweeps (as lbm_step, one parameter set,
 * one launch per step) reading the 16-bit codes of lbm_compress_adjacency:
 * a tile without escapes moves 19 * 2 * sizeof(PDF) + 36.3 bytes per cell
 * update instead of 19 * 2 * sizeof(PDF) + 72; a tile with escapes reads
 * adj.  The gathered slots are the ones adj names, so results are bitwise
 * equal to lbm_step's.
 *
 *  codes, tile_records  from lbm_compress_adjacency for the same n, stride
 *        and adj (other codes can address memory outside f).
 *  adj   the uncompressed list (read in tiles with escapes).
 *  ns, f_a, f_b, n_steps, stream  as lbm_step (f_a: state in; the result is
 *        in f_b after an odd, in f_a after an even number of steps).
 * Errors: LBM_EINVAL, LBM_EOVERFLOW, LBM_EHIP.
 */
lbm_status lbm_step_c16(const lbm_params* p, int64_t n, int64_t stride, const int16_t* codes,
                        const int32_t* tile_records, const uint32_t* adj, const double* ns,
                        void* f_a, void* f_b, int32_t n_steps, void* stream);

/*
 * lbm_narrow_codes -- 8-bit form of the 16-bit codes where a whole tile
 * allows it (further byte reduction of the adjacency read by the pull
 * updates of Sec. 7 over the list of Sec. 2).
 *
 * A tile (256 cells) is narrow when every code of its live cells is a
 * bounce-back (-32768) or lies in [-127, 127]; a tile with escapes never is.
 * For a narrow tile codes8[k * stride + m] = codes[k * stride + m], with
 * -128 for bounce-back, against the same per-tile offsets, and
 * tile_records[t * 20 + 19] is set to 1; for any other tile it is set to 0
 * and its codes8 entries to 0.
 *
 *  codes         int16 [18][stride] from lbm_compress_adjacency (input).
 *  tile_records  int32 [ceil(n / 256) * 20] from the same call (word 19 of
 *        every record is written).
 *  codes8        int8  [18][stride] (output; columns >= n untouched).
 *  n_narrow_tiles (host) number of narrow tiles.
 *  workspace, ws_bytes  2056 bytes of device scratch for partial sums
 *        (query with workspace NULL).  The call synchronizes the stream to
 *        return n_narrow_tiles.
 * Errors: LBM_EINVAL (NULL pointers, n <= 0), LBM_EOVERFLOW, LBM_EWORKSPACE,
 * LBM_EHIP.
 */
lbm_status lbm_narrow_codes(int64_t n, int64_t stride, const int16_t* codes,
                            int32_t* tile_records, int8_t* codes8, int64_t* n_narrow_tiles,
                            void* workspace, size_t* ws_bytes, void* stream);

/*
 * lbm_step_c8 -- lbm_step_c16 that reads codes8 in narrow tiles: such a tile
 * moves 19 * 2 * sizeof(PDF) + 18.3 bytes per cell update.  Other tiles read
 * the 16-bit codes, tiles with escapes adj.  Results are bitwise equal to
 * lbm_step's.
 *
 *  codes8, codes, tile_records  from lbm_narrow_codes and
 *        lbm_compress_adjacency for the same n, stride and adj.
 *  adj, ns, f_a, f_b, n_steps, stream  as lbm_step_c16.
 * Errors: LBM_EINVAL, LBM_EOVERFLOW, LBM_EHIP.
 */
lbm_status lbm_step_c8(const lbm_params* p, int64_t n, int64_t stride, const int8_t* codes8,
                       const int16_t* codes, const int32_t* tile_records, const uint32_t* adj,
                       const double* ns, void* f_a, void* f_b, int32_t n_steps, void* stream);

/*
 * lbm_step_inplace -- n_steps TRT pull sweeps on ONE PDF array (halves the
 * PDF memory of lbm_step's two arrays; the sweep of Sec. 7 on the sparse
 * representation of Sec. 2).
 *
 * Two kinds of step alternate.  Phase 0 ("layout P", the layout lbm_init and
 * lbm_step produce: slot (i, m) holds the post-collision f*_i of cell m):
 * each cell gathers through adj as lbm_step does, collides, and stores out_i
 * into the slot it gathered direction opp(i) from.  Phase 1 ("layout Q":
 * slot (opp(i), m) holds the population arriving at m in direction i): each
 * cell reads its own column with rows swapped, collides and stores out_i to
 * (i, m).  Each cell reads and writes the same 19 slots, so a step is safe in
 * place.  After an even number of steps from phase 0 the array is bitwise
 * what lbm_step gives; a tile of 256 cells moves 19 * 2 PDFs per step and
 * reads the adjacency only in phase-0 steps.
 *
 *  adj       the pull adjacency of lbm_build_adjacency.  The n listed cells
 *            must hold whole geometries: every slot adj names for m < n is a
 *            slot of a cell < n.
 *  codes, tile_records  16-bit codes of lbm_compress_adjacency for the same
 *            n, stride and adj (read instead of adj in phase-0 steps), or
 *            both NULL.
 *  ns        PBB solid fraction [stride] or NULL.
 *  f         [19][stride] state in layout `phase`; on return it is in layout
 *            (phase + n_steps) % 2.  lbm_moments and lbm_step expect layout P.
 *  phase     0 or 1.
 * Errors: LBM_EINVAL (bad params, NULL adj/f, phase not 0/1, only one of
 * codes and tile_records given), LBM_EOVERFLOW, LBM_EHIP.
 */
lbm_status lbm_step_inplace(const lbm_params* p, int64_t n, int64_t stride, const uint32_t* adj,
                            const int16_t* codes, const int32_t* tile_records, const double* ns,
                            void* f, int32_t phase, int32_t n_steps, void* stream);

/*
 * lbm_step_inplace_c8 -- lbm_step_inplace whose phase-0 steps read the 8-bit
 * codes of lbm_narrow_codes in narrow tiles, the 16-bit codes in the other
 * tiles and adj in tiles with escapes (the same byte reduction of the
 * adjacency read by the Sec. 7 pull updates as lbm_step_c8).  Results are
 * bitwise those of lbm_step_inplace.
 *
 *  codes8, codes, tile_records  from lbm_narrow_codes and
 *        lbm_compress_adjacency for the same n, stride and adj (all three
 *        required).
 *  The other arguments as lbm_step_inplace.
 * Errors: LBM_EINVAL (bad params, NULL pointers, phase not 0/1),
 * LBM_EOVERFLOW, LBM_EHIP.
 */
lbm_status lbm_step_inplace_c8(const lbm_params* p, int64_t n, int64_t stride,
                               const uint32_t* adj, const int8_t* codes8, const int16_t* codes,
                               const int32_t* tile_records, const double* ns, void* f,
                               int32_t phase, int32_t n_steps, void* stream);

/* Library version (major*10000 + minor*100 + patch) and a static string for a
 * status code.  Both are host-only and allocate nothing. */
int32_t lbm_version(void);
const char* lbm_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
