/*
 * hisq.h -- C ABI of libhisq.so: the improved-staggered (HISQ) Dslash and the
 * even-odd conjugate-gradient solves it drives, on one AMD MI355X (gfx950).
 *
 * Paper: R. Li, S. Gottlieb, "Staggered Dslash Performance on Intel Xeon Phi
 * Architecture", Lattice 2014.  Sec. 3 defines the operator's per-site work
 * (for each of the 8 directions +-mu a one-link "fat" matrix times the
 * nearest neighbour and a three-link "long" matrix times the third-nearest
 * neighbour: 16 matrix-vector products and 15 vector sums, 1146 flops) and
 * puts it inside single-mass and multi-shift CG; Sec. 4 solves on one parity
 * (even-odd preconditioning) with the staggered phases folded into the links.
 *
 * Conventions shared by every call
 *   dims[4]   = {Lx, Ly, Lz, Lt}; each extent even and >= 4, else HISQ_EDIMS.
 *             V = Lx*Ly*Lz*Lt sites, Vh = V/2 sites per parity.
 *   sites     lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) mod 2.
 *   vectors   one parity, [h][color] complex, h = lex >> 1 (Vh x 3 complex).
 *             complex128 (interleaved double re, im) for HISQ_F64,
 *             complex64 (interleaved float) for HISQ_F32 and HISQ_F16S.
 *   canonical links (input of hisq_pack_links): complex128
 *             [mu = x,y,z,t][lex][row][col], staggered phases and the time
 *             boundary sign already folded in (Sec. 4 absorbs the phases into
 *             the gauge field), so the library indexes periodically.
 *   operator  (D psi)(n) = sum_mu F_mu(n) psi(n+mu) - F_mu(n-mu)^dag psi(n-mu)
 *                               + L_mu(n) psi(n+3mu) - L_mu(n-3mu)^dag psi(n-3mu)
 *             (no factor 1/2); M = 2m + D; the even-odd system is
 *             A x_e = b_e with A = 4 m^2 - D_eo D_oe, Hermitian positive definite.
 *
 * Memory: every pointer argument that names a field is DEVICE memory owned by
 * the caller (for instance a torch tensor's data_ptr()); the library never
 * frees caller memory and does not allocate device memory on the solve path:
 * solvers take a caller-provided workspace sized by hisq_workspace_bytes().
 * The kernels read fields, links and workspaces with 16-byte loads: every
 * device pointer must be 16-byte aligned (device allocations are 256-byte
 * aligned), else HISQ_EINVAL.
 * `stream` is a hipStream_t (NULL = the null stream).  Calls are asynchronous
 * on `stream` except the solvers, which return when the solve has finished.
 *
 * Errors: every int-returning call returns HISQ_OK (0) or a negative
 * hisq_status; hisq_last_error() gives a message (thread-local, valid until
 * the next call on the same thread).  Errors of asynchronous GPU work surface
 * at the next synchronising call as HISQ_EHIP.  No C++ exception crosses the
 * ABI.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HISQ_OK = 0,
    HISQ_EINVAL = -1,      /* bad argument (NULL pointer, bad enum, bad size) */
    HISQ_EDIMS = -2,       /* a lattice extent is odd or < 4 */
    HISQ_EALIAS = -3,      /* an output buffer aliases an input */
    HISQ_EHIP = -4,        /* HIP runtime error */
    HISQ_ENOCONV = -5,     /* max_iter reached before tol (x holds the last iterate) */
    HISQ_EBREAKDOWN = -6,  /* <p, A p> <= 0 or not finite */
    HISQ_EWORKSPACE = -7   /* workspace NULL or smaller than hisq_workspace_bytes() */
} hisq_status;

/* Storage precision of links and vectors.
 * HISQ_F64  : FP64 links and vectors.
 * HISQ_F32  : FP32 links and vectors.
 * HISQ_F16S : FP16 links with one FP32 scale per (site, direction, field)
 *             matrix (the largest |re|, |im| of its 18 reals), FP32 vectors.
 * HISQ_I16S : 16-bit fixed-point links with the same per-matrix FP32 scale
 *             (entry = q * scale / 32767), FP32 vectors; same 40 B per matrix
 *             as HISQ_F16S with finer steps.
 * HISQ_F64C : FP64 with the long links in two-row form: rows 0 and 1 stored,
 *             row 2 rebuilt as c conj(row0 x row1), c = det = +-1 kept as a
 *             bit (Sec. 4: compression of the three-link term; the smeared
 *             fat links stay full).  Packing checks that every long link is
 *             +-SU(3) to 1e-6 and fails with HISQ_EINVAL otherwise.
 * HISQ_F32C : FP32 with two-row long links.
 * HISQ_I16SC: HISQ_I16S fat links and two-row long links in the same 16-bit
 *             fixed point (rows 0 and 1 with one FP32 scale per matrix).
 * HISQ_F32, HISQ_F16S, HISQ_I16S, HISQ_F32C and HISQ_I16SC have FP32
 * (complex64) vectors. */
typedef enum {
    HISQ_F64 = 0,
    HISQ_F32 = 1,
    HISQ_F16S = 2,
    HISQ_I16S = 3,
    HISQ_F64C = 4,
    HISQ_F32C = 5,
    HISQ_I16SC = 6
} hisq_prec;

/* CG modes.
 * PLAIN_F64  : every step in FP64.
 * MIXED_F32  : FP32 Dslash and vector updates inside, FP64 dot-product
 *              accumulation, FP64 reliable updates of the true residual
 *              (x += x_inner, r = b - A x in FP64) and FP64 final residual.
 * MIXED_F16S : as MIXED_F32 with HISQ_F16S links in the inner Dslash.
 * MIXED_I16S : as MIXED_F32 with HISQ_I16S links in the inner Dslash.
 * PLAIN_F64C : PLAIN_F64 with HISQ_F64C links.
 * MIXED_F32C : MIXED_F32 with HISQ_F64C outer and HISQ_F32C inner links.
 * MIXED_I16SC: MIXED_F32 with HISQ_F64C outer and HISQ_I16SC inner links.
 * Every mixed mode watches for stagnation: two reliable updates in a row
 * that do not reduce the true residual by a factor sqrt(delta) (by half when
 * delta < 0.25), or an inner solve that runs ten times
 * as long as its first cycle (plus 1000 iterations) without triggering an
 * update, end the mixed iteration; x then absorbs the inner solution and
 * plain CG on the outer links finishes the solve (stats.fallback_used = 1). */
enum {
    HISQ_CG_PLAIN_F64 = 0,
    HISQ_CG_MIXED_F32 = 1,
    HISQ_CG_MIXED_F16S = 2,
    HISQ_CG_MIXED_I16S = 3,
    HISQ_CG_PLAIN_F64C = 4,
    HISQ_CG_MIXED_F32C = 5,
    HISQ_CG_MIXED_I16SC = 6
};

/* cg_solve_multi modes.
 * MULTI_RHS   : nrhs independent systems A(m_i) x_i = b_i, one source and
 *               one mass each, advancing together: every Dslash application
 *               is one launch for all of them (each link load serves every
 *               right-hand side).
 * MULTI_SHIFT : one source b, nrhs masses: A(m_i) x_i = b, solved together
 *               by shifted CG (one Dslash pair per iteration for all shifts)
 *               on the inner links to opts->shift_tol (default max(tol, 1e-3)),
 *               then each x_i refined to tol by the batched reliable-update CG
 *               (skipped when opts->shift_only is set). */
enum { HISQ_MULTI_RHS = 0, HISQ_MULTI_SHIFT = 1 };

typedef struct {
    int mode;          /* HISQ_CG_* */
    int max_iter;      /* iteration cap over the whole solve (default 100000 if <= 0) */
    int check_every;   /* iterations between host convergence checks (<= 0: automatic) */
    int use_graph;     /* 1: replay check_every iterations as one captured HIP graph;
                          0: launch every kernel directly; 2 (cg_solve, plain modes):
                          direct launches timed with HIP events, see stats.kernel_us */
    double delta;      /* reliable-update trigger |r| < delta * max|r|, below 1 (>= 1 is
                          HISQ_EINVAL; <= 0: 0.7 for the 16-bit inner links F16S,
                          I16S, I16SC; 0.1 otherwise) */
    double shift_tol;  /* cg_solve_multi, MULTI_SHIFT: shift i leaves the shifted-CG phase
                          when its recursive residual |zeta_i r| / |b| <= shift_tol
                          (<= 0: max(tol, 1e-3); >= 1 is HISQ_EINVAL).  Ignored elsewhere */
    int shift_only;    /* cg_solve_multi, MULTI_SHIFT: 1 = return the shifted-CG solutions
                          as they are, without the batched refinement; stats[i] then
                          holds shift i's shifted-CG iterations, its recursive residual
                          (iter_resid) and the FP64 true residual of x_i, and status
                          HISQ_OK when the recursion reached shift_tol within max_iter
                          (HISQ_ENOCONV otherwise).  0 = refine to tol.  Ignored elsewhere */
} hisq_cg_opts;

typedef struct {
    int iters;              /* CG iterations (sloppy iterations for mixed modes) */
    int reliable_updates;   /* FP64 true-residual recomputations */
    int restarts;           /* plain mode: restarts after a failed final check */
    int status;             /* hisq_status of this solve */
    double true_resid;      /* |b - A x| / |b| recomputed in FP64 on the GPU */
    double time_s;          /* wall time of the solve, first kernel to final check */
    int fallback_used;      /* fcg_solve: 0 none; 1 K not positive on r or <p,Ap> <= 0; 2 too slow;
                               3 recursion converged but the true residual did not.
                               cg_solve mixed modes: 0 none; 1 stagnation, finished by plain CG */
    int fallback_iters;     /* plain CG iterations after the fallback (included in iters) */
    double iter_resid;      /* |r| / |b| of the solver's own recursion when it stopped (the
                               inner residual of a mixed solve; |zeta_i r| / |b| of a shift) */
    double bytes_moved;     /* algorithmic HBM bytes of the solve: every Dslash at its bytes per
                               site (links once, source once, output once) and every vector
                               stream once, summed over iterations and reliable updates
                               (cg_solve_multi: the whole batched solve, in every stats[i]) */
    double kernel_us[3];    /* cg_solve plain modes with opts->use_graph == 2: mean duration in
                               microseconds of the iteration's three main kernels, timed with
                               HIP events on the solve's stream: [0] t = D_oe p with the |t|^2
                               partials, [1] the parity-0 Dslash with A p in registers and the
                               x, r updates, [2] p = r + beta p with |p|^2; 0 otherwise */
} hisq_cg_stats;

/* Library version string. */
const char *hisq_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *hisq_last_error(void);

/* Bytes to allocate for EACH packed link field (fat and long; the larger of
 * the two for the compressed precisions) in precision `prec`, or 0 on bad
 * arguments.  The packed form stores, for every site of each parity and
 * for each of the 8 directions +-mu, the matrix that multiplies the
 * neighbour: F_mu(n) for +mu and -F_mu(n-mu)^dag for -mu (Sec. 4 stores
 * forward and backward links at every site for locality), in 64-site tiles
 * ordered [parity][tile][direction][element plane][site in tile]. */
size_t hisq_packed_link_bytes(const int dims[4], int prec);

/* Pack canonical links (device, complex128, layout above) into the packed
 * form of `prec` at fat_out / long_out (device, hisq_packed_link_bytes()
 * each).  `hop` of the fat field is 1 and of the long field 3 (Sec. 3: one-
 * and three-link terms).  Asynchronous on `stream`, except for the two-row
 * forms HISQ_F64C, HISQ_F32C and HISQ_I16SC, which synchronise to report
 * HISQ_EINVAL when a long link is not +-SU(3). */
int hisq_pack_links(const void *fat_canon, const void *long_canon, const int dims[4], int prec, void *fat_out,
                    void *long_out, void *stream);

/* dst = D src on the sites of parity `parity` (src lives on 1 - parity):
 * the Sec. 3 operator with 16 link matrices and 16 neighbour vectors per
 * site.  fat/lng: packed links of precision `prec`; src/dst: Vh x 3 complex
 * vectors of that precision's vector type.  src == dst -> HISQ_EALIAS.
 * Asynchronous on `stream`. */
int dslash_apply(const void *fat, const void *lng, const void *src, void *dst, int parity, const int dims[4],
                 int prec, void *stream);

/* y = A x = 4 m^2 x - D_eo (D_oe x) on the even sites (Sec. 4 even-odd
 * system).  tmp: Vh x 3 vector scratch (odd sites).  x, y, tmp distinct.
 * Asynchronous on `stream`. */
int hisq_apply_A(double mass, const void *fat, const void *lng, const void *x, void *y, void *tmp,
                 const int dims[4], int prec, void *stream);

/* Deterministic FP64 reductions over n complex entries of precision `prec`
 * vectors (Sec. 3: the dot products of CG): out_host[0] = Re <x, y>,
 * out_host[1] = Im <x, y> (y == x gives |x|^2).  Fixed order: wave64 tree,
 * per-workgroup partials (at most 1024 workgroups, striding over the
 * vectors), one fixed final sum; results are bitwise reproducible.
 * workspace: device scratch of hisq_workspace_bytes("dot", ...) bytes
 * (16.25 KB whatever n is), else HISQ_EWORKSPACE.  Synchronises `stream`. */
int hisq_dot(const void *x, const void *y, long long n, int prec, double out_host[2], void *workspace,
             size_t ws_bytes, void *stream);

/* hisq_dot without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the same two
 * kernels and result, on the library's own scratch, a static device array of
 * 16.25 KB per GPU (the first stage's at most 1024 partial pairs and the
 * result) held until the process ends.  Every call on a GPU uses that GPU's
 * one array: calls that overlap on one GPU race.  Any n from 0 to 2^37
 * complex entries (larger is HISQ_EINVAL); the scratch never grows with n.
 * Synchronises `stream`. */
int hisq_dot_noalloc(const void *x, const void *y, long long n, int prec, double out_host[2], void *stream);

/* Autotuner of the single-RHS Dslash launch shape (threads per workgroup,
 * occupancy target): times every shape with HIP events on the caller's
 * buffers (dst = D src on parity 1, `reps` launches each, 20 if <= 0),
 * remembers the fastest for (dims, prec) in this process -- and in the file
 * named by the environment variable HISQ_TUNE_CACHE, if set -- and uses it
 * in every later Dslash of that lattice and precision.  The plain CG's fused
 * kernels take the tile order of the chosen shape; for HISQ_F64 a shape with
 * a blocked tile order is chosen only when it is more than 3 % faster than
 * the fastest plain-order shape (the blocked orders slow the CG solve down
 * although the bare Dslash times them close to the plain one).  All shapes give
 * bitwise-identical results.  best_shape (may be NULL) receives the chosen
 * index, us_per_shape (may be NULL, room for hisq_dslash_shape(dims, prec,
 * -2) entries) the measured microseconds.  Synchronises `stream`. */
int hisq_tune_dslash(const void *fat, const void *lng, const void *src, void *dst, const int dims[4], int prec,
                     int reps, int *best_shape, double *us_per_shape, void *stream);

/* Launch shape of the single-RHS Dslash for (dims, prec): shape >= 0 sets
 * it, shape == -1 only queries; returns the shape in use, or a negative
 * hisq_status.  shape == -2 returns the number of shapes. */
int hisq_dslash_shape(const int dims[4], int prec, int shape);

/* Workspace bytes for `solver` = "cg", "cg_multi", "fcg", "fat_paths" or
 * "dot" on `dims` with `nrhs` right-hand sides (1 for cg), `mode` (HISQ_CG_*
 * for cg/fcg, HISQ_MULTI_* for cg_multi) and `channels` (fcg only);
 * fat_paths and dot ignore the last three.  0 on bad arguments. */
size_t hisq_workspace_bytes(const char *solver, const int dims[4], int nrhs, int mode, int channels);

/* Solve A(mass) x = b on the even sites to |b - A x| <= tol |b| (Sec. 3 CG;
 * Sec. 4 even-odd).  fat/lng: HISQ_F64 packed links (HISQ_F64C for the
 * PLAIN_F64C, MIXED_F32C and MIXED_I16SC modes).  fat_lo/lng_lo: HISQ_F32,
 * HISQ_F16S, HISQ_I16S, HISQ_F32C or HISQ_I16SC packed links matching the
 * mode, NULL for the plain modes.  b, x: complex128 Vh x 3; x holds x0 on
 * entry and the solution on exit (also on HISQ_ENOCONV).  opts NULL = plain
 * FP64 defaults.  stats (may be NULL) is always written.  Returns when the
 * solve has finished. */
int cg_solve(double mass, double tol, const void *fat, const void *lng, const void *fat_lo, const void *lng_lo,
             const void *b, void *x, const int dims[4], const hisq_cg_opts *opts, void *workspace,
             size_t ws_bytes, hisq_cg_stats *stats, void *stream);

/* Batched solves for nrhs <= 16 masses (Sec. 3: multishift CG over 9 or 11
 * masses).  masses: host array [nrhs], each > 0.  b: complex128
 * [nrhs][Vh][3] (MULTI_RHS) or [Vh][3] (MULTI_SHIFT); x: complex128
 * [nrhs][Vh][3], solved from x0 = 0 to |b_i - A(m_i) x_i| <= tol |b_i| for
 * every i.  fat/lng: F64 packed links (reliable updates, final residuals);
 * fat_lo/lng_lo: F32 packed links (inner iterations) for opts->mode
 * HISQ_CG_PLAIN_F64 or HISQ_CG_MIXED_F32; I16S for HISQ_CG_MIXED_I16S; for
 * HISQ_CG_MIXED_F32C and HISQ_CG_MIXED_I16SC, fat/lng are F64C and
 * fat_lo/lng_lo F32C or I16SC packed links (two-row long links, Sec. 4);
 * MIXED_F16S is HISQ_EINVAL.  opts: max_iter, check_every, use_graph and
 * delta as for cg_solve (default 0.7 for the 16-bit inner links, 0.1
 * otherwise).
 * stats: host array [nrhs] (may be NULL), per right-hand side; iters counts
 * the shifted-CG iterations plus the refinement iterations.  Returns
 * HISQ_ENOCONV / HISQ_EBREAKDOWN if any right-hand side failed; x then holds
 * every right-hand side's last iterate. */
int cg_solve_multi(int nrhs, const double *masses, double tol, int mode, const void *fat, const void *lng,
                   const void *fat_lo, const void *lng_lo, const void *b, void *x, const int dims[4],
                   const hisq_cg_opts *opts, void *workspace, size_t ws_bytes, hisq_cg_stats *stats,
                   void *stream);

/* Multi-RHS FP32 Dslash, the kernel inside the batched solver (Sec. 3
 * operator applied to nrhs vectors with one pass over the links): dst = D src
 * on parity `parity` for nrhs = 1, 2, 4, 8 or 16 right-hand sides stored
 * site-major, complex64 [Vh][nrhs][3].  fat/lng: HISQ_F32 packed links.
 * workspace: >= 4096 bytes of device memory (holds the launch's RHS mask).
 * Uses the launch shape chosen by hisq_tune_multi.  Asynchronous. */
int hisq_dslash_multi(const void *fat, const void *lng, const void *src, void *dst, int parity, int nrhs,
                      const int dims[4], void *workspace, size_t ws_bytes, void *stream);

/* Autotuner of the multi-RHS Dslash launch shape (right-hand sides per
 * thread, threads per workgroup) for (dims, nrhs): times every shape with
 * HIP events on the caller's buffers (as for hisq_dslash_multi, parity 1,
 * `reps` launches each) and remembers the fastest for hisq_dslash_multi.
 * cg_solve_multi chooses its own shape once per (dims, inner links, batch
 * size), timing its iteration's two launches, whose update epilogue needs
 * more registers per right-hand side.  us_per_shape (may be NULL) gets
 * hisq_multi_shape(dims, nrhs, -2) entries
 * (-1 for shapes that do not apply to nrhs).  Synchronises `stream`. */
int hisq_tune_multi(const void *fat, const void *lng, const void *src, void *dst, const int dims[4], int nrhs,
                    void *workspace, size_t ws_bytes, int reps, int *best_shape, double *us_per_shape,
                    void *stream);

/* ---- learned preconditioner ------------------------------------------------
 * A gauge-covariant linear network of four parallel-transport layers with
 * channels 1 -> C -> C -> C -> 1 (C = 4, 8 or 16):
 *     out^a(x) = sum_b sum_{k=0..8} W_k^{ab} (T_k in^b)(x),
 * T_0 = 1, T_{+mu} phi(x) = F_mu(x) phi(x+mu), T_{-mu} phi(x) =
 * F_mu(x-mu)^dag phi(x-mu), F the fat links of the operator (Sec. 3).  The
 * channel mixing runs on BF16 MFMA with FP32 accumulation, features are FP32;
 * the C -> 1 layer instead mixes the C channels at each neighbour in FP32 and
 * transports the one result (sum_k T_k sum_c W_k^c in^c, the same map).
 * Weights: complex64, the four layers' [9][C_out][C_in] arrays back to back
 * (net_weight_count() complex numbers).  Fields: complex64.  An even-site
 * input [batch][Vh][3] is embedded on the full lattice (odd sites zero); the
 * output is the even part of the last layer, [batch][Vh][3].  fat: the
 * HISQ_F32 packed fat links. */
size_t net_weight_count(int channels);
/* bytes of the activation buffer of net_forward (every layer's input is kept
 * for net_backward) and of net_backward's workspace.  Activation layout: four
 * BF16 weight-operand slots of 18432 bytes (the fourth unused), then the inputs of layers 1..4
 * and the output of layer 4, each [batch][channels][parity][Vh][3]
 * complex64 (1, C, C, C and 1 channels), every block starting at a multiple
 * of 256 bytes from the buffer's start. */
size_t net_act_bytes(const int dims[4], int channels, int batch);
size_t net_backward_ws_bytes(const int dims[4], int channels, int batch);
int net_forward(const void *fat, const void *weights, int channels, const void *in, void *out, void *acts,
                size_t act_bytes, int batch, const int dims[4], void *stream);
/* grad_out: dl/d out [batch][Vh][3]; grad_w: dl/dW summed over the batch
 * (complex, dl/dRe + i dl/dIm); grad_in (may be NULL): dl/d in.  acts: the
 * buffer filled by the net_forward of the same batch.  Layers 4, 3 and 2 take
 * their weight gradient from the transports of the upstream gradient g that
 * their input gradient computes anyway (sum_x <T_k x, g> = sum_x <x, T_{adj k} g>),
 * layer 1 from the transports of its one-channel input.  On return the
 * workspace starts with the gradients with respect to the input of layers 4,
 * 3 and 2 ([batch][channels][parity][Vh][3] complex64 each), then the
 * embedded grad_out and the gradient with respect to the input of layer 1
 * ([batch][1][parity][Vh][3] each, the latter written only when grad_in is
 * given), every block at a multiple of 256 bytes; the rest is scratch. */
int net_backward(const void *fat, const void *weights, int channels, const void *acts, size_t act_bytes,
                 const void *grad_out, void *grad_w, void *grad_in, int batch, const int dims[4], void *workspace,
                 size_t ws_bytes, void *stream);
/* The transported fields that the layers mix: out[b][k][c] = T_k in[b][c]
 * on the full lattice for k = 0..8 (k = 0 the identity, 1..4 the hops along
 * +x, +y, +z, +t, 5..8 along -x, -y, -z, -t), in FP32 from the same device
 * code as the layer kernels, which round exactly these values to BF16 for the
 * MFMA (the backward ones negated, with negated weights: the same products).  in: [batch][channels][parity][Vh][3] complex64 (channels 1, 4, 8 or
 * 16); out: [batch][9][channels][parity][Vh][3] complex64.  Asynchronous. */
int net_transport(const void *fat, const void *in, void *out, int channels, int batch, const int dims[4],
                  void *stream);
/* l = mean_b |y_b - x_b|^2 / |x_b|^2 (FP64 accumulation) into *loss_host
 * (may be NULL: no synchronisation) and dl/dy into grad_y (may be NULL).
 * workspace >= 2048 * (batch + 1) bytes. */
int net_loss(const void *y, const void *x, int batch, const int dims[4], double *loss_host, void *grad_y,
             void *workspace, size_t ws_bytes, void *stream);
/* Adam (Kingma & Ba 2014, beta1 0.9, beta2 0.999, eps 1e-8) on the real and
 * imaginary parts of n_complex weights; m, v: FP32 state of 2 n_complex
 * reals each, zero before step 1; step counts from 1. */
int net_adam_step(void *weights, const void *grad_w, void *m, void *v, long long n_complex, double lr, int step,
                  void *stream);
/* Flexible CG (Notay 2000, one stored direction, Polak-Ribiere update)
 * preconditioned by the network, on A(mass) x = b to tol; plain FP64 CG from
 * the current x is the fallback when K is not positive on the residual, when
 * <p, A p> <= 0, or when the lowest |r| reached over a window of 1000
 * iterations is not below half the lowest before it (stats.fallback_used
 * says which).  fat/lng: HISQ_F64 packed links; fat32:
 * HISQ_F32 packed fat links for the network.  Workspace from
 * hisq_workspace_bytes("fcg", dims, 1, 0, channels). */
int fcg_solve(double mass, double tol, const void *fat, const void *lng, const void *fat32, const void *weights,
              int channels, const void *b, void *x, const int dims[4], const hisq_cg_opts *opts, void *workspace,
              size_t ws_bytes, hisq_cg_stats *stats, void *stream);

/* ------------------------------------------------------------------ link construction
 * Sec. 4 of the paper: the three-link matrices of the Naik term are products
 * of thin links (matrix-matrix work).  Fields here are canonical complex128
 * [mu][t][z][y][x][3][3] device arrays (4 V matrices, 576 V bytes), periodic
 * indexing, no phases; hisq_fold_links then folds the staggered phases and
 * the time boundary sign in, and hisq_pack_links packs the result for the
 * Dslash.  All three are asynchronous on `stream`. */

/* out_mu(n) = U_mu(n) U_mu(n+mu) U_mu(n+2mu) for every site n and direction
 * mu.  out must not overlap thin (HISQ_EALIAS). */
int hisq_three_link(const void *thin, void *out, const int dims[4], void *stream);

/* Path-summed (smeared) one-link matrices from thin links U:
 *   out_mu(n) = coeff[0] U_mu(n) + coeff[1] S3 + coeff[2] S5 + coeff[3] S7 + coeff[4] SL,
 * each S the sum of the link products along every path of its family from n
 * to n+mu, over every direction nu != mu and both signs: 3-staples
 * U_nu(n) U_mu(n+nu) U_nu(n+mu)^dag and their mirror images (6 paths),
 * 5-staples (a 3-staple in rho around a 3-staple in nu, rho != nu: 24),
 * 7-staples (one more distinct axis: 48) and Lepage paths (a 3-staple
 * around a 3-staple in the same nu with the same sign: 6).  The weights are
 * inputs: the paper does not fix them.  workspace: device memory of
 * hisq_workspace_bytes("fat_paths", dims, 0, 0, 0) bytes (three one-direction
 * link fields).  out must not overlap thin or the workspace. */
int hisq_fat_paths(const void *thin, const double coeff[5], void *out, const int dims[4], void *workspace,
                   size_t ws_bytes, void *stream);

/* In place: links_mu(n) *= eta_mu(n) b_mu(n), with the staggered phases
 * eta_x = 1, eta_y = (-1)^x, eta_z = (-1)^(x+y), eta_t = (-1)^(x+y+z), and
 * b = -1 on the t-links whose hop of `hop` sites (1 for one-link, 3 for
 * three-link matrices) crosses the last time slice when antiperiodic_t is
 * nonzero, else 1.  HISQ_EINVAL unless hop is 1 or 3. */
int hisq_fold_links(void *links, const int dims[4], int hop, int antiperiodic_t, void *stream);

/* Measurement aid: microseconds per pass of a stream of nontemporal 16-byte
 * loads over `bytes` of device memory at `buf` (the load style of the Dslash's
 * link stream, 8 loads in flight per thread), averaged over `reps` passes after
 * one warm-up; the achievable HBM read rate that bounds every Dslash form.
 * sink: device scratch of >= 65536 bytes (block sums, so no load is dropped).
 * Synchronises `stream`. */
int hisq_read_probe(const void *buf, size_t bytes, void *sink, size_t sink_bytes, int reps, double *us,
                    void *stream);

/* Launch shape of the multi-RHS Dslash for (dims, nrhs): shape >= 0 sets it
 * (HISQ_EINVAL if it does not apply to nrhs), -1 queries, -2 returns the
 * number of shapes.  Returns the shape in use or a negative hisq_status. */
int hisq_multi_shape(const int dims[4], int nrhs, int shape);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
