/*
 * toeplitz.h - C ABI of the MI355X (gfx950) library that applies and solves the
 * impedance matrix of an Nx x Ny array of identical, electrically connected
 * elements (arXiv 2506.04710).
 *
 * The operator is Z = [[A, B^T], [B, C]] of eq. (matrixForm): A couples the
 * N = Nx*Ny*b element basis functions and is two-level block Toeplitz
 * (eq. submatrixAA), so it is fully described by the generator blocks Z_{m,n}
 * for offsets m in (-Nx, Nx), n in (-Ny, Ny); B and C couple the Nr rim (margin)
 * basis functions of Sec. II-B and are stored dense.  Nt = N + Nr.
 *
 * Vector ordering (Sec. II-C part order, x fastest): unknown (iy*Nx + ix)*b + p
 * is basis p of element (ix, iy); unknown N + r is rim function r.
 *
 * Conventions for every entry point:
 *   - complex numbers are interleaved (re, im); complex128 = 2 doubles,
 *     complex64 = 2 floats;
 *   - multi-vector arguments are column-major Nt x nrhs with a leading dimension
 *     ld >= Nt (column r starts at element r*ld);
 *   - a void* hip_stream is a hipStream_t (NULL = the default stream);
 *   - arguments are validated before any device work; a bad argument returns
 *     TP_E_INVAL and leaves every buffer untouched;
 *   - no call throws, aborts or allocates device memory: the plan lives in a
 *     device buffer the caller owns (e.g. a torch tensor);
 *   - after a non-OK status, toeplitz_last_error() returns a message for the
 *     calling thread.
 */
#ifndef TOEPLITZ_H
#define TOEPLITZ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tp_plan_s *tp_plan; /* opaque; host-side metadata owned by the library */

typedef enum {
    TP_OK = 0,
    TP_E_INVAL = 1,       /* invalid argument (shape, pointer, size, option) */
    TP_E_NOMEM = 2,       /* the caller's device buffer is smaller than toeplitz_plan_bytes() */
    TP_E_HIP = 3,         /* a HIP runtime call failed; the message names it */
    TP_E_NOCONV = 4,      /* a solve column missed its tolerance within the iteration limits */
    TP_E_BREAKDOWN = 5,   /* Krylov breakdown without convergence (e.g. singular operator) */
    TP_E_UNSUPPORTED = 6  /* valid request this build does not handle (e.g. missing precision copy) */
} tp_status;

/* Which operator copies a plan holds, and which one a matvec uses. */
typedef enum {
    TP_FP64 = 0,   /* complex128 spectrum and rim, FP64 arithmetic */
    TP_FP32 = 1,   /* complex64 spectrum and rim, FP32 arithmetic with FP32 accumulation */
    TP_MIXED = 2,  /* both copies (plans); for solves: FP32 operator inside FP64 refinement */
    /* range markers, not precisions: every int is a value of the type, so an
       out-of-range argument reaches the library's check (TP_E_INVAL) */
    TP_PREC_RANGE_MIN_ = -2147483647 - 1,
    TP_PREC_RANGE_MAX_ = 2147483647
} tp_prec;

/* Plan layout facts, filled by toeplitz_plan_info. */
typedef struct {
    int Nx, Ny, b, Nr;
    int Px, Py;              /* circulant grid, Px >= 2Nx-1, Py >= 2Ny-1 */
    long N, Nt;
    int max_rhs, restart;
    tp_prec prec;
    size_t spectrum_bytes;   /* per copy: Px*Py*b*b complex values, or (Px/2+1)*Py*b*b with half_spectrum */
    size_t rim_bytes;        /* per copy: B (Nr x N), optional B_er^T (Nr x N), C (Nr x Nr) */
    size_t workspace_bytes;  /* FFT grids, partial sums and the Krylov workspace */
    size_t total_bytes;      /* == toeplitz_plan_bytes() */
    int reciprocal;          /* 1 if the element-rim block is rim_re transposed */
    int half_spectrum;       /* 1 if the generators are symmetric and half the spectrum is stored */
    int nrc;                 /* rim channels per cell of a placed rim (toeplitz_plan_create_placed), else 0 */
    int bc;                  /* channels per cell of the transforms and spectrum blocks: b + nrc */
} tp_plan_desc;

/*
 * Symmetry of the operator (the impedance matrix is symmetric, Sec. II-B), as
 * bits of the sym argument of toeplitz_plan_bytes:
 *   TP_SYM_RIM  the element-rim block is rim_re transposed (rim_er NULL): one
 *               dense rim block per precision instead of two;
 *   TP_SYM_GEN  the generators satisfy Z_{-m,-n} = Z_{m,n}^T: then the
 *               spectrum satisfies Ghat(-k) = Ghat(k)^T and the plan stores
 *               only the columns kx <= Px/2 (about half the spectrum bytes,
 *               and half the spectrum stream of every matvec).
 */
#define TP_SYM_RIM 1
#define TP_SYM_GEN 2

/*
 * Device bytes a plan needs: the operator copies selected by prec (spectrum of
 * the generators, Sec. I / eq. submatrixAA, plus the dense rim of eqs.
 * submatrixBB..submatrixC456), FFT grids for up to max_rhs columns and the
 * Krylov workspace of GMRES(restart) for max_rhs columns.  Use it for admission
 * before creating a plan.  sym: TP_SYM_RIM when rim_er will be NULL, plus
 * TP_SYM_GEN when toeplitz_gen_symmetric reports the generators symmetric
 * (toeplitz_plan_create decides the same way).  bytes receives the size;
 * returns TP_E_INVAL for Nx, Ny, b < 1, Nr < 0, max_rhs < 1, restart < 1, Nx or
 * Ny > 256, b > 256, Nr > 2048, restart > 512, unknown sym bits or sizes that
 * overflow.
 */
tp_status toeplitz_plan_bytes(int Nx, int Ny, int b, int Nr, int sym, tp_prec prec,
                              int max_rhs, int restart, size_t *bytes);

/*
 * Host check of the generator symmetry Z_{-m,-n} = Z_{m,n}^T (Sec. II-B):
 * *symmetric = 1 if gen[2Ny-2-n][2Nx-2-m][q][p] equals gen[n][m][p][q] bit for
 * bit for every entry, else 0.  gen: host complex128 in the layout of
 * toeplitz_plan_create.  Errors: TP_E_INVAL (NULL pointers, Nx, Ny, b outside
 * [1, 256]).
 */
tp_status toeplitz_gen_symmetric(int Nx, int Ny, int b, const double *gen, int *symmetric);

/*
 * Build a plan in the caller's device buffer (Sec. II-C structure; Sec. I FFT
 * route): the generators are circulant-embedded in a Px x Py grid, transformed
 * by a 2-D DFT (forward sign exp(-2 pi i k n / P)) and scaled by 1/(Px Py); the
 * rim blocks are copied.  Symmetric generators (toeplitz_gen_symmetric) keep
 * only the spectrum columns kx <= Px/2; the others are applied as transposes.  Every host input is copied; the caller may free them
 * on return.  The call synchronises hip_stream before returning.
 *
 *   gen     host complex128 [2Ny-1][2Nx-1][b][b] with
 *           gen[n+Ny-1][m+Nx-1][p][q] = Z_{m,n}[p][q], the block between basis p
 *           of element (ix+m, iy+n) (row) and basis q of element (ix, iy).
 *   rim_re  host complex128 [Nr][N]: rim row r, element column e (NULL iff Nr = 0).
 *   rim_er  host complex128 [N][Nr]: element row e, rim column r; NULL means the
 *           reciprocal case rim_er[e][r] = rim_re[r][e] (Sec. II-A symmetry).
 *   rim_rr  host complex128 [Nr][Nr] (NULL iff Nr = 0).
 *   dev_buf device buffer of dev_bytes >= toeplitz_plan_bytes(...) bytes, 256-byte
 *           aligned; owned by the caller, who must keep it alive until
 *           toeplitz_plan_destroy and free it afterwards.
 *   out     receives the plan handle.
 * Errors: TP_E_INVAL (shapes, NULL pointers, misaligned buffer, a NaN or Inf
 * in gen or a rim block), TP_E_NOMEM
 * (dev_bytes below toeplitz_plan_bytes with the sym bits this call implies),
 * TP_E_HIP.
 */
tp_status toeplitz_plan_create(int Nx, int Ny, int b, int Nr, const double *gen,
                               const double *rim_re, const double *rim_er, const double *rim_rr,
                               tp_prec prec, int max_rhs, int restart, void *dev_buf,
                               size_t dev_bytes, void *hip_stream, tp_plan *out);

/*
 * Structured rim (the margin decomposition of Sec. II-B and the one-level
 * block-Toeplitz rim blocks of eqs. submatrixB12, submatrixB34, submatrixC123,
 * submatrixC456): every rim function belongs to a margin part that repeats by
 * translation with the elements, so it can be pinned to an element cell with
 * a fixed local offset.  Then every coupling of Z, rim included, depends only
 * on the difference of the two cells, and Z is the restriction, to the
 * occupied (cell, channel) pairs, of one two-level block-Toeplitz operator with
 * bc = b + nrc channels per cell.  A placed plan stores the spectrum of that
 * operator (no dense B or C) and applies the whole of Z with the element
 * kernels: the embedding scatters x_r into the rim channels of their cells and
 * the crop gathers y_r from them.
 *
 * toeplitz_plan_bytes_placed: as toeplitz_plan_bytes for a placed rim with
 *   nrc >= 1 rim channels per cell (TP_SYM_GEN when the extended generators
 *   are symmetric, which holds for symmetric generators with a reciprocal rim
 *   and a symmetric rim_rr).
 * toeplitz_plan_create_placed: as toeplitz_plan_create, plus
 *   rim_place  host int [Nr][3]: rim function r sits at element cell
 *              (rim_place[r][0], rim_place[r][1]) in [0, Nx) x [0, Ny) as
 *              channel b + rim_place[r][2], rim_place[r][2] in [0, nrc); no
 *              two functions share a cell and channel.  (A margin part outside
 *              the cell range is placed at the nearest cell: its whole
 *              component moves with it, which changes no coupling.)
 *   The extended generators are assembled on the host from gen, rim_re,
 *   rim_er (or rim_re transposed) and rim_rr; every entry must receive the same
 *   value, bit for bit, from every pair of rim/element functions whose cells
 *   have that offset.  Errors: as toeplitz_plan_create, plus TP_E_INVAL when
 *   the placement is out of range or shared, or the rim blocks are not block
 *   Toeplitz in it (checked before any device work).  A placed plan has no
 *   rim elimination (toeplitz_schur_* return TP_E_UNSUPPORTED); its
 *   preconditioner inverts the extended spectrum blocks, rim channels included.
 */
tp_status toeplitz_plan_bytes_placed(int Nx, int Ny, int b, int Nr, int nrc, int sym, tp_prec prec,
                                     int max_rhs, int restart, size_t *bytes);
tp_status toeplitz_plan_create_placed(int Nx, int Ny, int b, int Nr, const double *gen,
                                      const double *rim_re, const double *rim_er, const double *rim_rr,
                                      const int *rim_place, int nrc, tp_prec prec, int max_rhs,
                                      int restart, void *dev_buf, size_t dev_bytes, void *hip_stream,
                                      tp_plan *out);

/*
 * Launch options of a plan: kernel variants that compute the same result
 * (bit for bit within one option value) at different speeds on different
 * shapes; the tuner (toeplitz_tune) measures them and sets the fastest.
 *   TP_OPT_SPECTRUM_PASS  one column without a dense rim pass over a half
 *     spectrum (the preconditioner, and the operator of a placed rim):
 *     TP_PASS_FUSED  one launch per column chunk that transforms along y,
 *                    streams the stored blocks and transforms back;
 *     TP_PASS_PAIRS  y transforms in passes of their own and a stream that
 *                    reads each stored block once in its own workgroup and
 *                    applies it to its frequency and, transposed, to the
 *                    mirror frequency;
 *     TP_PASS_AUTO   (default) the fused launch.
 *   TP_OPT_MFMA_COLS  columns per workgroup of the matrix-core product (16,
 *     32 or 64, FP64 products take at most 32; 0 = default: 16 up to 16
 *     columns, else 32 for FP32 and 16 for FP64).
 *   TP_OPT_MFMA_MIN_R  number of columns from which products and the dense rim
 *     pass run on the matrix cores (2..max_rhs; 0 = default 16).
 *   TP_OPT_FFT2_LDS  LDS bytes a workgroup of the 2-D transform tiles may take
 *     (16384..163840; 0 = default 49152): grids whose tile of 4 channels fits
 *     run both transform directions in one launch instead of two passes.
 *   TP_OPT_MULTI_FUSED  1: 16+ columns on a grid of 2-D tiles run every stage
 *     (dense reciprocal rim slabs, forward tiles, matrix-core products,
 *     inverse tiles, rim finish) in one persistent launch whose workgroups
 *     take tasks from a queue in dependency order (same results bit for bit);
 *     0 (default): one launch per stage.  Applies with even b, the default
 *     column tile, no separate B_er and TP_OPT_PROD_LDS off.
 *   TP_OPT_RIM_OVERLAP  1 (default): where the dense rim runs on the matrix
 *     cores and the transforms on 2-D tiles (16+ columns on small grids), the
 *     rim's slabs and the forward tiles share one launch (independent work: the
 *     rim's matrix work overlaps the transforms); 0: two launches.  Same
 *     results bit for bit.
 *   TP_OPT_DUAL_LAUNCH  1 (default): a mixed solve (TP_MIXED) applies its
 *     FP32 operator (Arnoldi steps) and its FP64 operator (residual steps) in
 *     shared launches, one per stage, where both precisions take the same
 *     launch shape: one column on the pair-stream path with separate x and y
 *     passes, or many columns with the matrix-core product at its default
 *     column tiles (TP_OPT_MFMA_COLS 0, TP_OPT_PROD_LDS 0, no persistent
 *     launch) on separate passes or on 2-D tiles, without a dense rim pass
 *     (the idle instance costs no launch of its own); with the
 *     preconditioner on one column, its last pass (inverse x transforms) and
 *     the operator's first (forward x transforms) also share one launch; 0:
 *     one launch sequence per precision.  Same results bit for bit.
 *   TP_OPT_PROD_LDS  FP32 per-frequency product with the spectrum block staged
 *     in LDS and each wave's column tile of the transformed input held in
 *     registers: value 16 * CG + RT (+ 256), CG column tiles of 16 per
 *     workgroup (1..15), RT row tiles of 16 per wave (2, 3 or 6); + 256 (half
 *     spectrum): one workgroup per stored block, applied to its frequency and
 *     transposed to the mirror frequency, so each stored block is read once;
 *     0 (default): the product that streams the block from memory.  Same
 *     results bit for bit; applies from the matrix-core column threshold on,
 *     to b <= 128, where CG * ceil(ceil(b / 16) / RT) <= 16 (else the
 *     default product runs).
 * Setting an option drops the plan's captured solver graphs.  Errors:
 * TP_E_INVAL (unknown option or value, NULL pointers, a continuous batch is
 * active on the plan).
 */
#define TP_OPT_SPECTRUM_PASS 1
#define TP_OPT_MFMA_COLS 2
#define TP_OPT_MFMA_MIN_R 3
#define TP_OPT_FFT2_LDS 4
#define TP_OPT_MULTI_FUSED 5
#define TP_OPT_PROD_LDS 6
#define TP_OPT_RIM_OVERLAP 7
#define TP_OPT_DUAL_LAUNCH 8
#define TP_PASS_AUTO 0
#define TP_PASS_FUSED 1
#define TP_PASS_PAIRS 2
tp_status toeplitz_plan_set_option(tp_plan p, int option, int value);
tp_status toeplitz_plan_get_option(tp_plan p, int option, int *value);

/*
 * Which launches an application takes (a description, for tuning and tests):
 * the operator (precond = 0) or the preconditioner (precond = 1) in precision
 * `which` (as toeplitz_matvec) at nrhs columns, with the plan's current
 * options.  Sets *flags to an OR of
 *   TP_PATH_FUSED       one column, fused spectrum pass (transforms in it)
 *   TP_PATH_PAIRS       one column, pair-stream spectrum pass
 *   TP_PATH_MFMA        products on the matrix cores (many columns)
 *   TP_PATH_DENSE_RIM   a dense rim pass (operator of a plan without a placed rim)
 *   TP_PATH_RIM_MFMA    that rim pass on the matrix cores
 *   TP_PATH_TILES2D     both transform directions per launch on 2-D tiles
 *   TP_PATH_PERSISTENT  every stage in one persistent launch (TP_OPT_MULTI_FUSED)
 *   TP_PATH_RIM_OVERLAP the rim's slabs and the forward tiles in one launch
 *                       (TP_OPT_RIM_OVERLAP)
 *   TP_PATH_JOINED      (which = TP_MIXED, precond = 1, nrhs = 1) a mixed
 *                       solve's preconditioner inverse x pass and operator
 *                       forward x pass share one launch (TP_OPT_DUAL_LAUNCH)
 * Launches nothing.  Errors: TP_E_INVAL (NULL plan or flags, bad precision,
 * nrhs outside [1, max_rhs], precond without a preconditioner),
 * TP_E_UNSUPPORTED (the plan lacks the copy `which` needs).
 */
#define TP_PATH_FUSED 1
#define TP_PATH_PAIRS 2
#define TP_PATH_MFMA 4
#define TP_PATH_DENSE_RIM 8
#define TP_PATH_RIM_MFMA 16
#define TP_PATH_TILES2D 32
#define TP_PATH_PERSISTENT 64
#define TP_PATH_RIM_OVERLAP 128
#define TP_PATH_JOINED 256
tp_status toeplitz_plan_path(tp_plan p, tp_prec which, int precond, int nrhs, int *flags);

/* Result of toeplitz_tune: the options it set and the time they gave. */
typedef struct {
    int spectrum_pass;   /* TP_PASS_FUSED or TP_PASS_PAIRS (TP_PASS_AUTO when no launch depends on it) */
    int mfma_cols;       /* 16, 32, 64 (0 when nrhs is below the matrix-core threshold) */
    int fft2_lds;        /* 0 (48 KB tiles) or 163840 (where larger tiles would change the path) */
    int multi_fused;     /* 1 where the persistent multi-column launch was timed and fastest, else 0 */
    int prod_lds;        /* TP_OPT_PROD_LDS value chosen (0: the streaming product) */
    int rim_overlap;     /* TP_OPT_RIM_OVERLAP value chosen */
    int candidates;      /* option combinations timed */
    double ms;           /* mean milliseconds of the timed work with the chosen options */
    double ms_default;   /* the same with every option at its default */
} tp_tune_result;

/*
 * Autotuner: time every combination of the launch options that changes a
 * kernel on this plan at nrhs columns (the spectrum pass for one column over
 * a half spectrum without a dense rim pass: placed-rim operators and the
 * preconditioner; the matrix-core column tile from the threshold on; the 2-D
 * transform tile size where a 160 KB tile of 4 channels would hold a grid
 * that a 48 KB one does not; the persistent multi-column launch where a
 * combination at the default column tile takes it; for FP32 operators from
 * the threshold on, the LDS-staged product in column-group and row-tile
 * shapes whose workgroup fits; the rim and forward tiles in one launch or
 * two where that applies), each
 * for reps applications after two untimed ones, with HIP events on
 * hip_stream, and set the fastest.  The timed work is what a solve applies:
 * the operator `which` (TP_FP64, TP_FP32 or TP_MIXED, as toeplitz_matvec) and,
 * if the plan has a preconditioner, its application in the same precision.
 * x, y: device work vectors as for toeplitz_matvec (any content; y is
 * overwritten).  Synchronises hip_stream.  Errors: as toeplitz_matvec,
 * TP_E_INVAL for reps < 1 or a NULL result.
 */
tp_status toeplitz_tune(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                        int reps, void *hip_stream, tp_tune_result *result);

/* Copy the plan's layout facts into *desc. */
tp_status toeplitz_plan_info(tp_plan p, tp_plan_desc *desc);

/*
 * y = Z x for nrhs columns (eq. MoMMatrixEq operator): embed, forward 2-D DFT,
 * per-frequency b x b block product with the stored spectrum, inverse DFT, crop,
 * plus the dense rim terms y_A += B_er x_r, y_r = B x_A + C x_r.
 * x, y: device, column-major Nt x nrhs, leading dimensions ldx, ldy >= Nt.
 * which selects the operator copy and the vector type:
 *   TP_FP64   FP64 operator, complex128 vectors;
 *   TP_FP32   FP32 operator (FP32 accumulation), complex64 vectors;
 *   TP_MIXED  FP32 operator on complex128 vectors (inputs rounded to FP32 as
 *             they are read, results widened as they are written): the inner
 *             operator of a TP_MIXED solve.
 * x and y must not overlap.  1 <= nrhs <= max_rhs.  Asynchronous on
 * hip_stream; uses the plan's workspace, so calls on one plan must not run
 * concurrently, and the call is refused (TP_E_INVAL) while a continuous batch
 * runs on the plan.
 * Errors: TP_E_INVAL, TP_E_UNSUPPORTED (the plan lacks that precision copy),
 * TP_E_HIP.
 */
tp_status toeplitz_matvec(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy,
                          int nrhs, void *hip_stream);

/*
 * For callers that cannot allocate or hand over workspace (code under HIP graph
 * capture, serving loops that forbid allocation): the same y = Z x as
 * toeplitz_matvec, same arguments, checks and kernels, but the transform grids,
 * rim slab partial sums and mirror parts live in a static device array of
 * toeplitz_static_scratch_bytes() bytes (64 MiB) that the library holds on each
 * device it runs on until the process ends, not in the plan's workspace.  The
 * call allocates nothing.  The workspace one call needs is
 * 2 * max(Ny*Px, Px*Py) * b * nrhs * 16 bytes of grids, plus
 * nslab * max(Nr, 1) * nrhs * 16 bytes of rim partials, plus, for a half
 * spectrum, (b/8) * Ny * (Px - kxh) * b * 16 bytes of mirror parts (each rounded
 * up to 256 bytes); a call that needs more returns TP_E_INVAL before any device
 * work.  Every call on a device shares that device's array and leaves its last
 * contents there: calls that overlap in time on one device (on any streams,
 * from any threads or plans) race and give wrong results; order them on one
 * stream.  The device of p must be current.
 * Errors: as toeplitz_matvec, plus TP_E_INVAL for a workspace beyond the limit.
 */
tp_status toeplitz_matvec_static(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy,
                                 int nrhs, void *hip_stream);
/* Size in bytes of the static workspace of toeplitz_matvec_static. */
size_t toeplitz_static_scratch_bytes(void);

/*
 * Instrumentation: run the operator application of toeplitz_matvec `reps`
 * times on hip_stream with HIP events between its kernels and write the mean
 * duration in milliseconds of each stage to stage_ms[7]: 0 rim pass over B,
 * 1 embed + x transform, 2 y transform, 3 per-frequency block product,
 * 4 inverse y transform, 5 inverse x transform + crop, 6 rim finish (C x_r).
 * Stages a plan does not run (no rim) report 0.  Same arguments and errors as
 * toeplitz_matvec; synchronises hip_stream.
 */
tp_status toeplitz_matvec_profile(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy,
                                  int nrhs, int reps, void *hip_stream, double *stage_ms);

/*
 * Instrumentation: the mean duration in milliseconds of one stage of the
 * operator application (numbered as in toeplitz_matvec_profile; 3 is the
 * per-frequency product, or the fused pass that includes it), launched reps
 * times back to back between two HIP events on hip_stream, after one full
 * application that leaves every stage's input in the plan's workspace (each
 * stage rewrites the same output from the same input, so the repeats are
 * alike).  No event sits between the repeats.  A stage the plan's path does
 * not have launches nothing.  Same arguments and errors as toeplitz_matvec,
 * plus TP_E_INVAL for a NULL ms, reps < 1 or a stage outside 0..5;
 * synchronises hip_stream.
 */
tp_status toeplitz_stage_time(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy,
                              int nrhs, int stage, int reps, void *hip_stream, double *ms);

/* Solver options (all fields are read; see toeplitz_solve_opts_default). */
typedef struct {
    double tol;        /* stop when ||v - Z x||_2 / ||v||_2 <= tol, FP64 residual */
    int restart;       /* GMRES restart length m (<= the plan's restart) */
    int max_iter;      /* cap on Arnoldi steps (operator applications) per column */
    int max_outer;     /* cap on refinement steps (TP_MIXED) or restarts (TP_FP64) */
    tp_prec mode;      /* TP_FP64: GMRES on the FP64 operator; TP_MIXED: FP32 inner GMRES
                          with FP64 residual refinement; TP_FP32 is not a solve mode */
    int x0_given;      /* 1: x holds the initial guess; 0: start from zero */
    double inner_tol;  /* TP_MIXED: relative residual target of each inner solve */
    int precond;       /* 1: right-precondition with the plan's block-circulant preconditioner
                          (toeplitz_precond_create); 0: none */
} tp_solve_opts;

/* Per-column result of toeplitz_solve. */
typedef struct {
    int iters;         /* Arnoldi steps (operator applications inside GMRES) */
    int outer_iters;   /* FP64 residual evaluations after the first */
    int status;        /* TP_OK, TP_E_NOCONV or TP_E_BREAKDOWN */
    double relres;     /* final ||v - Z x||_2 / ||v||_2 from an FP64 matvec */
} tp_solve_info;

/* Defaults: tol 1e-8, restart = plan's, max_iter 2000, max_outer 50, TP_FP64, x0 zero, inner_tol 1e-4,
   no preconditioner. */
void toeplitz_solve_opts_default(tp_solve_opts *opts);

/*
 * Solve Z x = v (eq. MoMMatrixEq) for nrhs columns with restarted GMRES
 * (Sec. II-D names GMRES on the second Toeplitz level; Arnoldi with classical
 * Gram-Schmidt and one reorthogonalisation, Givens QR of the Hessenberg matrix,
 * all in FP64 on the device).  Each column has its own Krylov space; columns
 * converge independently and stop on their own FP64 residual.
 * v, x: device complex128, column-major Nt x nrhs, ldv, ldx >= Nt, not
 * overlapping.  info: host array of nrhs entries, filled on return.
 * opts NULL = defaults.  The call synchronises hip_stream (the host reads the
 * convergence scalars).  Returns TP_OK if every column met tol, TP_E_NOCONV /
 * TP_E_BREAKDOWN otherwise (x then holds each column's best iterate and info is
 * filled), TP_E_INVAL / TP_E_UNSUPPORTED / TP_E_HIP on errors.  A column
 * whose right-hand side holds NaN or Inf stops at its first residual with
 * status TP_E_INVAL (the call then returns TP_E_INVAL with info filled; the
 * other columns run to their own end).  Solves are limited to Nt <= 262144
 * unknowns (TP_E_UNSUPPORTED beyond; the Krylov kernels keep two rounds of 256
 * elements per thread in registers for 512 element ranges).
 */
tp_status toeplitz_solve(tp_plan p, const void *v, long ldv, void *x, long ldx, int nrhs,
                         const tp_solve_opts *opts, tp_solve_info *info, void *hip_stream);

/*
 * Continuous batching (serving): a plan runs one GMRES engine with max_rhs
 * slots.  Each slot solves one column Z x = v independently (same method and
 * options as toeplitz_solve); columns are admitted into free slots and
 * released after they finish while the other slots keep iterating, so
 * requests that arrive while others are running join the running batch.
 * All work runs on the plan's own stream (default priority); the calls below
 * only enqueue work, except batch_poll with wait = 1 and batch_end.
 *
 * toeplitz_batch_begin: start the engine (opts as for toeplitz_solve; NULL =
 *   defaults); every slot starts idle.  Errors as toeplitz_solve.
 * toeplitz_batch_admit: put column v (device complex128, Nt contiguous values)
 *   into an idle or released slot; x (device complex128, Nt values) receives
 *   the solution (x0_given = 1: x holds the initial guess).  The engine waits
 *   for work already enqueued on hip_stream (so v may be written there).  v and
 *   x must stay valid until the slot is released.
 * toeplitz_batch_release: return a slot to idle (after it finished, or to
 *   cancel it).
 * toeplitz_batch_step: enqueue ngraphs rounds of two GMRES super-steps for
 *   all slots, then an asynchronous copy of the slot states.
 * toeplitz_batch_poll: slot states after the latest (lag = 0) or the previous
 *   (lag = 1) batch_step: phases[max_rhs] = 0 idle, 1 running, 2 finished, and
 *   info[max_rhs] (status/iters/relres, final once finished); with wait = 0
 *   returns TP_E_NOCONV if that step has not completed yet (no error).  Once a
 *   slot reads finished, its x is complete in device memory.
 * toeplitz_batch_end: wait for the engine's stream and stop the batch
 *   (toeplitz_solve is refused on the plan while a batch is active).
 */
tp_status toeplitz_batch_begin(tp_plan p, const tp_solve_opts *opts);
tp_status toeplitz_batch_admit(tp_plan p, int slot, const void *v, void *x, double tol, int x0_given,
                               void *hip_stream);
tp_status toeplitz_batch_release(tp_plan p, int slot);
tp_status toeplitz_batch_step(tp_plan p, int ngraphs);
tp_status toeplitz_batch_poll(tp_plan p, int lag, int wait, int *phases, tp_solve_info *info);
tp_status toeplitz_batch_end(tp_plan p);

/*
 * Schur-complement elimination of the rim (the solve structure of Sec. II-D on
 * eq. matrixForm): with Z = [[A, B_er], [B, C]],
 *   setup  F = A^-1 B_er (Nr solves with the element operator A alone),
 *          S = C - B F and its inverse;
 *   solve  w = A^-1 v_A,  x_r = S^-1 (v_r - B w),  x_A = w - F x_r,
 * so the iterated operator is the two-level block-Toeplitz A.  `a` is a plan of
 * the same array (same Nx, Ny, b and generators) with Nr = 0: it supplies A and
 * runs the Toeplitz solves (its preconditioner, if opts->precond).  The plan p
 * must hold the FP64 operator.  The caller owns the buffer (dev_bytes >=
 * toeplitz_schur_bytes, 256-byte aligned) and keeps it until p is destroyed.
 * toeplitz_schur_create synchronises hip_stream; the element solves use opts
 * (mode, tol, precond, ...) and may return TP_E_NOCONV.  Errors: TP_E_INVAL,
 * TP_E_NOMEM, TP_E_UNSUPPORTED, TP_E_BREAKDOWN (S singular), TP_E_HIP.
 */
tp_status toeplitz_schur_bytes(tp_plan p, size_t *bytes);
tp_status toeplitz_schur_create(tp_plan p, tp_plan a, void *dev_buf, size_t dev_bytes,
                                const tp_solve_opts *opts, void *hip_stream);

/*
 * Solve Z x = v through the elimination built by toeplitz_schur_create.  v, x:
 * device complex128, column-major Nt x nrhs (ld >= Nt), 1 <= nrhs <= max_rhs of
 * both plans.  The element solves run to opts->tol / 2; info[r].relres is the
 * true ||v - Z x|| / ||v|| of the full system from an FP64 application, and
 * status TP_OK when it is <= opts->tol (else TP_E_NOCONV, x holds the result);
 * iters and outer_iters are those of the element solve.  Synchronises hip_stream.
 * Refused (TP_E_INVAL) while a continuous batch runs on either plan.
 */
tp_status toeplitz_schur_solve(tp_plan p, tp_plan a, const void *v, long ldv, void *x, long ldx, int nrhs,
                               const tp_solve_opts *opts, tp_solve_info *info, void *hip_stream);

/*
 * Copy one block of the stored spectrum to the host (the bc x bc matrix at
 * frequency (kx, ky), row-major, bc = b, or b + nrc for a placed rim (the
 * extended generators); host_out holds bc * bc complex128 for TP_FP64,
 * complex64 for TP_FP32).
 * It equals (1/(Px Py)) sum_{m,n} Z_{m,n} exp(-2 pi i (kx m / Px + ky n / Py)).
 * Synchronous.  Errors: TP_E_INVAL, TP_E_UNSUPPORTED, TP_E_HIP.
 */
tp_status toeplitz_plan_spectrum(tp_plan p, tp_prec which, int kx, int ky, void *host_out);

/*
 * Block-circulant preconditioner (the paper gives none; Sec. II-D leaves the
 * solver's details to another reference).  With C_P the block circulant of the
 * generators placed on the plan's Px x Py grid (the embedding the operator uses),
 *   M^-1 x = [ crop(C_P^-1 pad(x_A)) ; x_r / diag(C) ],
 * applied as an inverse DFT of S(k) DFT(pad x_A) with S(k) = (sum of the
 * placed generators times exp(-2 pi i (kx m / Px + ky n / Py)))^-1 per
 * frequency.  GMRES then solves Z M^-1 u = v and returns x = M^-1 u (right
 * preconditioning: the residual it tests is the true one).
 *
 * toeplitz_precond_bytes: device bytes the preconditioner of this plan needs
 *   (S per precision the plan holds, 1/diag(C), a status word).
 * toeplitz_precond_create: build it into dev_buf (caller-owned, >= that many
 *   bytes, 256-byte aligned, kept until toeplitz_plan_destroy) by inverting
 *   every b x b frequency block in FP64 (Gauss-Jordan, partial pivoting).
 *   Needs a plan with the FP64 copy (TP_FP64 or TP_MIXED; else
 *   TP_E_UNSUPPORTED).  Synchronises hip_stream; a singular block or a zero
 *   diagonal entry of C returns TP_E_BREAKDOWN.  A second call rebuilds (and
 *   drops the plan's captured solver graphs, which hold the old pointers);
 *   refused while a continuous batch runs on the plan.
 * toeplitz_precond_bytes_for: the same count before a plan exists (for
 *   admission), from the arguments of toeplitz_plan_bytes (sym as there;
 *   prec TP_FP64 or TP_MIXED, else TP_E_UNSUPPORTED).
 * toeplitz_precond_apply: y = M^-1 x for nrhs columns (same conventions as
 *   toeplitz_matvec, including which = TP_MIXED: the FP32 copy on complex128
 *   vectors, as a mixed solve applies it; x and y must not overlap).
 *   TP_E_INVAL without a preconditioner.  Asynchronous on hip_stream.
 */
tp_status toeplitz_precond_bytes(tp_plan p, size_t *bytes);
tp_status toeplitz_precond_bytes_for(int Nx, int Ny, int b, int Nr, int sym, tp_prec prec, size_t *bytes);
tp_status toeplitz_precond_create(tp_plan p, void *dev_buf, size_t dev_bytes, void *hip_stream);
tp_status toeplitz_precond_apply(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                                 void *hip_stream);

/*
 * Post-steps on solved currents (Sec. III; they need no plan).
 *
 * toeplitz_port_smatrix: scattering matrix of p ports from the p solutions of
 * the port excitations (Sec. III-B): column j of X (device complex128, Nt
 * values per column, ld ldx >= Nt) is the current vector for a unit excitation
 * at port j; port_rows (host int64 [p], each in [0, Nt)) are the unknowns of
 * the ports, edge_len (host double [p], each > 0; NULL = all 1) their edge
 * lengths.  With I_hat[i][j] = X[port_rows[i], j], L = diag(1 / edge_len),
 * Y = L I_hat L and Z_port = Y^-1, the result is
 * S = (Z_port - Z0 I)(Z_port + Z0 I)^-1 (equal real reference impedance Z0 > 0
 * on every port), written column-major p x p to S (device complex128,
 * ld lds >= p).  It is computed as S = (I + Z0 Y)^-1 (I - Z0 Y), which equals
 * the definition whenever Y is invertible (both factors are functions of Y),
 * by Gaussian elimination with partial pivoting; no inverse is formed.
 * work: device scratch of work_bytes >= 32 p^2 + 16 p + 256 bytes, 8-byte
 * aligned.
 * 1 <= p <= 1024.  Synchronises hip_stream.  A zero pivot (I + Z0 Y singular)
 * returns TP_E_BREAKDOWN (S undefined).
 *
 * toeplitz_far_field: far field of nrhs current vectors by the per-part
 * contraction of eqs. (farfieldBasis) and (tensorProd), for point-dipole basis
 * functions: element basis n sits at u_n + (ix dx, iy dy, 0) with unit tangent
 * t_n (elem_pos, elem_tan: device double [b][3]); rim function r at c_r with
 * tangent t_r (rim_pos, rim_tan: device double [Nr][3], NULL if Nr = 0).  For
 * direction m (dirs: device double [nang][2] = (theta, phi) in radians),
 *   F_tau = -j k eta [ sum_e exp(j k rhat.d_e) sum_n I[e b + n] (e_tau.t_n) exp(j k rhat.u_n)
 *                      + sum_r I[N + r] (e_tau.t_r) exp(j k rhat.c_r) ],
 * e_theta = (cos th cos ph, cos th sin ph, -sin th), e_phi = (-sin ph, cos ph, 0).
 * I: device complex128, column-major Nt x nrhs (ld ldi).  F: device complex128
 * [nrhs][nang][2] (tau = theta, phi).  1 <= Nx, Ny, b <= 1024, Nr >= 0,
 * 1 <= nrhs <= 65535, nang >= 1.  Asynchronous on hip_stream.
 */
tp_status toeplitz_port_smatrix(int p, long Nt, const void *X, long ldx, const long *port_rows,
                                const double *edge_len, double Z0, void *S, long lds, void *work, size_t work_bytes,
                                void *hip_stream);
tp_status toeplitz_far_field(int Nx, int Ny, int b, int Nr, double dx, double dy, const double *elem_pos,
                             const double *elem_tan, const double *rim_pos, const double *rim_tan, const void *I,
                             long ldi, int nrhs, const double *dirs, int nang, double k, double eta, void *F,
                             void *hip_stream);

/* Release the plan's host metadata.  The caller frees dev_buf afterwards. NULL is ignored. */
void toeplitz_plan_destroy(tp_plan p);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *toeplitz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TOEPLITZ_H */
