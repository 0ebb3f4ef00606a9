/*
 * stiles.h -- C ABI of an MI355X (gfx950) FP64 library for the selected
 * inversion of symmetric positive-definite band-plus-arrowhead matrices.
 *
 * Method: arXiv 2504.19171 ("GPU-Accelerated Parallel Selected Inversion for
 * Structured Matrices Using sTiles"), Sec. III.  A = L L^T is factored on the
 * band and arrow tiles (the sTiles tile Cholesky the paper builds on, whose
 * kernels it names in Sec. III-F: POTRF/TRSM/SYRK/GEMM), and Sigma = A^{-1} is
 * computed only on the tile pattern of L ("case 7" of Sec. III-B) by the
 * two-phase backward recurrence of Sec. III-D (Phase 1: diagonal-tile inverse
 * and TRMM of each tile row; Phase 2: LAUUM and GEMM accumulations from the
 * bottom-right tile to the top-left one).  log det A = 2 sum_j log L_jj is
 * returned with the factor (not in the paper).
 *
 * Conventions common to every call
 * --------------------------------
 * - All matrices are IEEE binary64.  Sizes are int64_t.
 * - n is the total order, `arrow` (a) the number of dense trailing rows and
 *   columns, nb = n - a the order of the band part, `bandwidth` (w) the
 *   half-bandwidth of the band part in elements (w >= nb-1 means a dense band),
 *   `tile` (b) the tile size.  Constraints: n >= 1, 0 <= a < n, w >= 0,
 *   tile in {64, 128, 192, 256}, a <= 512.
 * - Tile layout ("tiles" below), one buffer of stiles_layout.total_doubles
 *   doubles, every tile column-major:
 *     band tile (J+d, J), J < N = ceil(nb/b), 0 <= d <= B:  b x b, leading
 *       dimension b, at off_band + (J*(B+1) + d) * b*b; B = min(ceil(w/b), N-1).
 *       Tiles with J+d >= N exist and are kept zero.
 *     arrow tile J (rows nb .. nb+a_p-1, tile column J):  a_p x b, leading
 *       dimension a_p, at off_arrow + J * a_p*b; a_p = a rounded up to 16.
 *     corner (rows and columns nb .. nb+a_p-1):  a_p x a_p, leading dimension
 *       a_p, at off_corner.
 *   Padding makes every tile full: band rows nb .. N*b-1 and arrow rows
 *   a .. a_p-1 are identity on the diagonal and zero elsewhere.  This is exact:
 *   Sigma on real indices and log det are unchanged (log 1 = 0).
 * - Pointers named "device" are HIP device pointers; the caller allocates and
 *   frees every buffer.  The library never retains or frees caller memory and
 *   allocates no device memory.
 * - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *   enqueues work on `stream` and returns; results are ready when the stream
 *   is.  Calls on different streams may overlap if they use different buffers
 *   and workspaces.  The library creates no streams or events of its own
 *   (except the timing events of stiles_timing_enable).
 * - Return value: 0 when the work was enqueued; -i when argument i (1-based)
 *   is invalid; STILES_EHIP when a HIP call failed.  Numerical outcomes are
 *   reported in the device `info` word (see stiles_factor / stiles_selinv).
 */
#ifndef STILES_H
#define STILES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STILES_OK 0
#define STILES_EHIP (-100)      /* a HIP runtime call failed */
#define STILES_ETIMEOUT (-101)  /* a device wait on a tile-ready flag exceeded its spin limit */
#define STILES_EBADL (-102)     /* stiles_selinv: a diagonal entry of L is not positive */
#define STILES_ENOTBUILT (-103) /* reserved for bindings: library not loaded */

typedef struct stiles_layout {
    int64_t n, bandwidth, arrow; /* arguments as given */
    int32_t tile;                /* b */
    int32_t bt;                  /* B: tile half-bandwidth */
    int64_t nb;                  /* n - arrow */
    int64_t w;                   /* min(bandwidth, nb - 1) */
    int64_t nt;                  /* N: band tile rows/columns */
    int32_t arrow_ld;            /* a_p: arrow rounded up to 16 (0 when arrow == 0) */
    int32_t reserved;
    int64_t off_band, off_arrow, off_corner; /* offsets in doubles */
    int64_t total_doubles;       /* size of one tile buffer in doubles */
} stiles_layout;

/*
 * Fill *out with the tile layout of a matrix (host only, no GPU call): this
 * library's form of the compressed tile format that the method keeps the
 * matrix in (selection step of Sec. III-B), for the arrowhead structure of
 * Sec. II-III (band tiles within B of the diagonal, the arrow rows as a tile
 * row of their own, the corner).  Returns 0, or -i for an invalid argument i.
 */
int stiles_layout_init(int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                       stiles_layout* out);

/*
 * Pack a matrix given in canonical band form (device memory, row-major) into
 * the tile layout (device memory), writing every double of `tiles`:
 *   ab     [(w+1) x nb]  ab[d*nb + j] = A[j+d][j], w = min(bandwidth, nb-1)
 *   arrow_rows [a x nb]  arrow_rows[r*nb + j] = A[nb+r][j]  (NULL if a == 0)
 *   corner [a x a]       corner[r*a + c] = A[nb+r][nb+c], full symmetric
 *                        (NULL if a == 0)
 * The paper stores the matrix in its "compressed tile format" shared with the
 * Cholesky (Sec. III-B, selection step); this call builds this library's
 * version of it.  Padding is written as described above.
 */
int stiles_pack(const double* ab, const double* arrow_rows, const double* corner,
                double* tiles, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                void* stream);

/* Workspace sizes in bytes (host only). */
size_t stiles_factor_workspace_bytes(const stiles_layout* lay);
size_t stiles_selinv_workspace_bytes(const stiles_layout* lay);

/*
 * Tile Cholesky A = L L^T on the band and arrow tiles, and log det A.
 *   A         device, tile layout, read only the lower triangles of diagonal
 *             tiles and of the corner.
 *   L         device, tile layout, output.  L may equal A (in place).  The
 *             upper triangles of the diagonal tiles and the corner are set to
 *             0; entries of band tiles outside the element band come out 0.
 *   logdet    device, one double: 2 * sum_j log L_jj (NaN if not SPD).
 *   info      device, one int32: 0 on success; k > 0 if the pivot of global
 *             column k (1-based, k <= n) is not positive or is NaN, as in
 *             LAPACK potrf -- L is then partly overwritten; STILES_ETIMEOUT if
 *             a device wait exceeded its spin limit.
 *   workspace device, at least stiles_factor_workspace_bytes(); contents on
 *             entry are ignored.
 * Defined by the problem statement of Sec. III (A SPD, A = L L^T) and the
 * tile kernels named in Sec. III-F.
 */
int stiles_factor(const double* A, double* L, int64_t n, int64_t bandwidth, int64_t arrow,
                  int32_t tile, double* logdet, int32_t* info, void* workspace,
                  size_t workspace_bytes, void* stream);

/*
 * Selected inverse: Sigma = A^{-1} on the tile pattern of L (Sec. III-B,
 * case 7), by Phase 1 and Phase 2 of Sec. III-D.
 *   L         device, tile layout, a factor produced by stiles_factor (read only).
 *   Sigma     device, tile layout, output: every band tile (J+d, J) with
 *             J+d < N, every arrow tile and the corner hold Sigma; diagonal
 *             tiles and the corner are full symmetric.  Must not alias L.
 *   info      device, one int32: 0 on success; STILES_EBADL if a diagonal
 *             entry of L is <= 0 or NaN; STILES_ETIMEOUT as above.
 *   workspace device, at least stiles_selinv_workspace_bytes().
 */
int stiles_selinv(const double* L, double* Sigma, int64_t n, int64_t bandwidth, int64_t arrow,
                  int32_t tile, int32_t* info, void* workspace, size_t workspace_bytes,
                  void* stream);

/*
 * Batched form: `count` independent matrices, each with its own n, bandwidth,
 * arrow and tile, factored (or inverted) together.  The paper treats one
 * matrix per call (Sec. III); here every launch of the single-matrix path
 * covers all the matrices that have work in it, each on its own share of the
 * workgroups with its own tickets and counters, so a batch of small matrices
 * fills the device.  The tasks and their arithmetic are those of stiles_factor
 * and stiles_selinv on each matrix alone: results are identical bit for bit.
 *
 * The factor's launches run in step across the batch: each covers eight
 * consecutive tile columns of every matrix that has them (the environment
 * variable STILES_KB_COLS, 1 to 16, sets the count; the columns of a launch
 * are chained through per-block update counters), so the batch takes about as
 * long as its longest matrix, and a batch with one tile size runs best.  With
 * every tile at most 128 wide, the factor runs two workgroups per compute unit.
 *
 * items (host array of `count` entries, read during the call only):
 *   n, bandwidth, arrow, tile   as for stiles_layout_init; reserved must be 0
 *   A       device, tile layout input of stiles_factor_batched
 *   L       device, L (output of the factor, input of the selinv); may equal A
 *   Sigma   device, Sigma output of stiles_selinv_batched (ignored by the
 *           factor); must not alias L
 *   logdet  device, one double (factor)
 *   info    device, two int32: [0] as stiles_factor's info, [1] as
 *           stiles_selinv's info
 * workspace  device, at least stiles_batch_workspace_bytes(items, count); one
 *           workspace serves both calls (contents on entry are ignored).
 * The calls copy a small table of the matrices into the workspace with
 * hipMemcpyAsync on `stream`, staged in pinned host memory that the library
 * owns (up to 16 buffers, kept until the process ends; a buffer is reused
 * once its copy has completed, and when all are busy the call waits for one).
 * The call returns without waiting for the copy itself.
 * Returns 0; -1 if items is NULL or an item is invalid (its layout, a NULL
 * pointer, reserved != 0, or for the selinv Sigma NULL or equal to L); -2 if
 * count < 1; -3 / -4 for the workspace and its size; STILES_EHIP.
 */
typedef struct stiles_batch_item {
    int64_t n, bandwidth, arrow;
    int32_t tile;
    int32_t reserved;
    const double* A;
    double* L;
    double* Sigma;
    double* logdet;
    int32_t* info;
} stiles_batch_item;

/* Workspace size in bytes for a batch (host only); 0 if an item is invalid. */
size_t stiles_batch_workspace_bytes(const stiles_batch_item* items, int32_t count);

/* stiles_factor on every item: L and log det of each matrix. */
int stiles_factor_batched(const stiles_batch_item* items, int32_t count, void* workspace,
                          size_t workspace_bytes, void* stream);

/* stiles_selinv on every item: Sigma on the tile pattern of each L. */
int stiles_selinv_batched(const stiles_batch_item* items, int32_t count, void* workspace,
                          size_t workspace_bytes, void* stream);

/*
 * The batched calls in two parts, for replay from a HIP graph (the batching
 * of the method's calls, as above): stiles_batch_upload copies the tables of
 * both calls for these items into their two areas of the workspace (staged
 * and stream-ordered like the calls above; items need Sigma set); the
 * _enqueue variants then only enqueue device work (kernels
 * and, where A != L, device-to-device copies) that reads those tables and
 * restarts every counter it uses, so a stream capture of them can be
 * replayed any number of times.  Each _enqueue call must be given the same
 * items, in the same order, as the upload that wrote the tables, and the
 * workspace must not be used for another batch in between.  Per-kernel
 * timing (stiles_timing_enable) must be off while a stream is captured.
 * Arguments and return values as for the calls above.
 */
int stiles_batch_upload(const stiles_batch_item* items, int32_t count, void* workspace,
                        size_t workspace_bytes, void* stream);
int stiles_factor_batched_enqueue(const stiles_batch_item* items, int32_t count, void* workspace,
                                  size_t workspace_bytes, void* stream);
int stiles_selinv_batched_enqueue(const stiles_batch_item* items, int32_t count, void* workspace,
                                  size_t workspace_bytes, void* stream);

/*
 * Selection (Sec. III-B, selection step and symbolic inversion).  A selected
 * (i, j) lies in tile column J (J = j / b in the band part, or the corner);
 * the recurrence for tile column J reads only tile columns to its right, so
 * the closure of a selection inside the tile pattern of L is every tile column
 * from the leftmost selected one to the last, and nothing to the left of it is
 * computed.
 *
 * stiles_selinv_range: stiles_selinv restricted to the tile columns
 *   J >= first_column (0 <= first_column <= N; N: the corner alone).  Those
 *   columns and the corner of Sigma come out as from stiles_selinv, bit for
 *   bit; the other band and arrow tiles of Sigma are left undefined.
 *   Arguments as stiles_selinv, with first_column as argument 7.
 * stiles_gather: out[k] = Sigma(ij[2k], ij[2k+1]) (either order) for count
 *   pairs (device arrays: ij int64 [2 count], out double [count]); NaN for a
 *   pair outside the tile pattern of L or outside the matrix.
 */
/*
 * stiles_selection_closure: the symbolic step of a selection, on the host
 *   (no device work).  For count pairs ij[2k], ij[2k+1] (host int64, either
 *   order, 0 <= index < n): *inside (host int32) = 1 when every pair lies in
 *   the tile pattern of L (a band pair whose tile row is at most B tiles below
 *   its tile column, or any pair with an arrow index), else 0;
 *   *first_column (host int64) = the leftmost tile column holding a selected
 *   pair (N when every pair lies in the corner, or count == 0).  When *inside
 *   is 1, stiles_selinv_range from *first_column followed by stiles_gather
 *   yields every selected entry; otherwise some pair needs entries outside
 *   the pattern (stiles_inverse).  Returns 0; -k for a bad argument k (-5
 *   also for a pair outside the matrix); nothing is written on an error.
 */
int stiles_selection_closure(int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile, const int64_t* ij,
                             int64_t count, int32_t* inside, int64_t* first_column);
int stiles_selinv_range(const double* L, double* Sigma, int64_t n, int64_t bandwidth, int64_t arrow,
                        int32_t tile, int64_t first_column, int32_t* info, void* workspace,
                        size_t workspace_bytes, void* stream);
int stiles_gather(const double* Sigma, int64_t n, int64_t bandwidth, int64_t arrow, int32_t tile,
                  const int64_t* ij, int64_t count, double* out, void* stream);

/*
 * Full inverse: every entry of A^{-1}, by the backward recurrence of Phase 2
 * (Sec. III-D) taken over all tile rows instead of the rows of S(J) -- the
 * full-inversion case of the selection spectrum (Sec. III-B) -- after Phase 1.
 * Dense output, so for modest n: the workspace holds a dense padded copy,
 * (N b + a_p)^2 doubles, and the work grows as n^2 (w + a).
 *   L         device, tile layout, a factor produced by stiles_factor (read only)
 *   Ainv      device, n x n column-major (leading dimension n), full symmetric
 *   info      device, one int32: 0, or STILES_EBADL as for stiles_selinv
 *   workspace device, at least stiles_inverse_workspace_bytes()
 */
size_t stiles_inverse_workspace_bytes(const stiles_layout* lay);
int stiles_inverse(const double* L, double* Ainv, int64_t n, int64_t bandwidth, int64_t arrow,
                   int32_t tile, int32_t* info, void* workspace, size_t workspace_bytes,
                   void* stream);

/*
 * Trace of a product on the tile pattern, for the gradient of log det:
 *   *out = sum_ij Sigma_ij B_ij  over the real entries (padding left out),
 * with Sigma and B symmetric and stored in the tile layout of one matrix,
 * Sigma as stiles_selinv writes it and B as stiles_pack writes it (diagonal
 * tiles and the corner full, band tiles below the diagonal and arrow tiles
 * standing for their mirrored upper parts too).  When the pattern of B lies
 * in the tile pattern of L this is tr(A^{-1} B); with B = dA/dtheta it is
 * d log det A / dtheta (Jacobi's formula; the paper's selected inverse is what
 * makes it cheap, Sec. I).  Fixed summation order: repeatable bit for bit.
 *   Sigma, B  device, tile layout (read only)
 *   out       device, one double
 *   workspace device, at least stiles_trace_workspace_bytes()
 */
size_t stiles_trace_workspace_bytes(void);
int stiles_trace_product(const double* Sigma, const double* B, int64_t n, int64_t bandwidth,
                         int64_t arrow, int32_t tile, double* out, void* workspace,
                         size_t workspace_bytes, void* stream);

/*
 * Per-kernel timing with HIP events (tracing support, not needed for results).
 * While enabled, every kernel the library enqueues is bracketed by a pair of
 * HIP events recorded on the same stream.  stiles_timing_collect() waits for
 * the recorded events, adds their durations per kernel kind into
 * ms[STILES_TK_COUNT] and launches[STILES_TK_COUNT] (host arrays, overwritten),
 * releases the events and starts a new collection.  Enabling or disabling
 * drops events not collected yet.  Thread-safe; costs two event records per
 * launch while enabled.
 */
#define STILES_TK_POTRF 0      /* factor: the corner's diagonal blocks (POTRF) */
#define STILES_TK_TRSM 1       /* factor: reserved (panel TRSM runs inside the tile-column launches) */
#define STILES_TK_UPDATE 2     /* factor: reserved (trailing updates run inside the tile-column launches) */
#define STILES_TK_PHASE1 3     /* selinv: Phase 1 (TRTRI, TRMM, LAUUM) */
#define STILES_TK_PHASE2 4     /* selinv: Phase 2 (persistent kernel) */
#define STILES_TK_FACTOR 5     /* factor: one launch per band tile column (POTRF + TRSM + updates) */
#define STILES_TK_OTHER 6      /* pack, copies, corner, finalization */
#define STILES_TK_COUNT 7
int stiles_timing_enable(int on);
int stiles_timing_collect(double* ms, int64_t* launches);

/*
 * Matrix-core throughput probe (measurement support, not part of the method):
 * enqueues one launch of 2 workgroups per compute unit in which every
 * wavefront issues `iters` x 8 independent FP64 16x16x4 matrix-core products,
 * and sets *flops (host) to the floating-point operations it performs, so
 * that flops / elapsed time is the FP64 matrix-core rate the device sustains.
 *   sink   device, at least 512 doubles per compute unit (results are junk,
 *          written only so the work is kept).
 * Returns -1 (sink too small or NULL), -3 (iters < 1), -4 (flops NULL), or
 * STILES_EHIP.
 */
int stiles_mfma_peak(double* sink, int64_t sink_doubles, int32_t iters, double* flops, void* stream);

/* Static text for a return or info code.  A positive code k is the LAPACK
 * potrf convention for the first non-positive pivot (the factor's diagonal
 * tile kernel is the POTRF named in Sec. III-F); the negative codes are the
 * argument and runtime errors listed above. */
const char* stiles_strerror(int code);

/* Library version, major*10000 + minor*100 + patch. */
int stiles_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STILES_H */
