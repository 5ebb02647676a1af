/*
 * flashmp.h - C ABI of the FlashMP hot path on one AMD Instinct MI355X (gfx950).
 *
 * The library solves the Crank-Nicolson FDTD double-curl system
 *     A E = b,   A = I + c diag(1/eps_e) K,   K = C^T C   (Sec. II-A, eqs. (4)-(5);
 *                                                         Sec. III-A, eqs. (6)-(7))
 * on Yee grids with PEC walls, preconditioned by restricted additive Schwarz
 * (Sec. II-B) whose subdomain solves are exact discrete-transform solves
 * (Sec. III-A, Steps 1-3; Algorithm 1, exact_solve): forward DCT-II/DST-I
 * transforms along x, y, z per staggered component, a closed-form 3x3 solve
 * per wavenumber (eq. (12)), inverse transforms.
 *
 * Vector layout (every vector argument):
 *   Device pointers to FP64 arrays.  One block per domain, concatenated at the
 *   offsets returned by fmp_vector_layout.  Inside a domain of nx*ny*nz cells
 *   the block is [3][nz][ny][nx] (components E_x, E_y, E_z; x fastest).
 *   E_x sits at (i+1/2, j, k) in slot [k][j][i]; E_y at (i, j+1/2, k) in
 *   [k][j][i]; E_z at (i, j, k+1/2) in [k][j][i].  Slot 0 along a component's
 *   two node axes is the PEC wall: ignored on input, written as 0 on output.
 *   The far wall node (index n) is not stored.
 *
 * Ownership: the caller owns every vector and every workspace.  A handle owns
 *   small host-side plans only; its device tables live in the setup workspace,
 *   which must stay allocated and untouched until fmp_destroy.  Nothing in
 *   this library allocates device memory.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  fmp_curlcurl_apply and fmp_apply_precond only enqueue work and
 *   are safe to capture in a hipGraph; fmp_solve synchronises the stream for
 *   its convergence checks.
 *
 * Errors: functions return an fmp_status; no exception crosses the ABI.  On a
 *   negative status no output has been written unless stated.  The detail of
 *   the last error on a handle is available from fmp_last_error.
 *
 * Threading: a handle is not thread safe; distinct handles are independent.
 * Determinism: FP64 reductions use a fixed order, so results are bitwise
 *   reproducible on one device for one configuration.
 */
#ifndef FLASHMP_H
#define FLASHMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmp_ctx* fmp_handle;

typedef enum {
  FMP_OK = 0,
  FMP_NOT_CONVERGED = 1,      /* result usable; see fmp_solve_info              */
  FMP_ERR_INVALID_ARG = -1,   /* bad descriptor, size or null pointer           */
  FMP_ERR_ALIAS = -2,         /* input and output vectors overlap               */
  FMP_ERR_WORKSPACE = -3,     /* workspace missing, too small or misaligned     */
  FMP_ERR_HIP = -4,           /* a HIP runtime call failed                       */
  FMP_ERR_BREAKDOWN = -5,     /* Krylov breakdown or non-finite value           */
  FMP_ERR_UNSUPPORTED = -6    /* valid request the library does not implement   */
} fmp_status;

typedef enum { FMP_FP64 = 0, FMP_FP32 = 1, FMP_BF16 = 2 } fmp_precision;

/* One domain: a box of nx*ny*nz unit cells with PEC walls on all six faces.
 * c = dt^2/(4 mu eps0 h^2) (the alpha of eq. (7) for eps_r = 1).
 * eps_block: host array of relative permittivities, one per cube of
 *   eps_block_size^3 cells, C order [ceil(nz/b)][ceil(ny/b)][ceil(nx/b)]
 *   (the library reads that many values); NULL means eps_r = 1.
 *   The permittivity at an E edge is the mean over the four cells sharing it.
 * sub_x/y/z: owned subdomain side in cells (must divide the domain side;
 *   0 = the whole axis, i.e. one box). */
typedef struct {
  int32_t nx, ny, nz;
  double c;
  const double* eps_block;
  int32_t eps_block_size;
  int32_t sub_x, sub_y, sub_z;
} fmp_domain_desc;

/* Preconditioner options.
 * overlap: Schwarz overlap gamma in cells, >= 1 (boxes are clipped at walls).
 * precision: arithmetic of the transforms and block solve (fmp_precision).
 *   FP64 and FP32 run on the vector ALU; BF16 runs the transforms as MFMA
 *   GEMMs on bf16 operands with FP32 accumulation.
 * use_learned: 1 reserves room for a coarse-correction network
 *   (fmp_set_coarse_model); it is applied only once weights are set.
 * batch_boxes: boxes per pipeline batch (0 = automatic); smaller batches keep
 *   the transform staging resident in the last-level cache.  -1 = automatic,
 *   and the workspace keeps room for every candidate of fmp_autotune.
 * use_graph: 1 = the launch sequence of an apply is captured once per
 *   (r, z) pair into a hipGraph (on a private stream, default priority) and
 *   replayed on the caller's stream; at most 64 pairs are cached, further
 *   pairs run uncaptured.  Results are identical to uncaptured applies.
 * subdomain: the subdomain of each Schwarz term.
 *   0 = PEC box (default): the unknowns strictly inside the owned block
 *       extended by `overlap` cells (overlap >= 1), one exact transform solve
 *       per box (Sec. III-A Steps 1-3).
 *   1 = index block (Sec. III-A Step 4; Algorithm 1 main body): the unknowns
 *       whose half-point and node indices lie in [a - overlap, a + n + overlap)
 *       along every axis, clipped at the grid (overlap >= 0).  Each apply
 *       runs two exact solves with the compact-difference bases around the
 *       low-rank boundary correction C^{-1} (one dense (6n^2-3n)^2 matrix per
 *       distinct box shape, wall pattern and alpha, built on the device at
 *       setup; 293 MB at n = 32).  FP64 only, sides <= 48, no learned part,
 *       no autotuner (FMP_ERR_UNSUPPORTED otherwise). */
typedef struct {
  int32_t overlap;
  int32_t precision;
  int32_t use_learned;
  int32_t batch_boxes;
  int32_t use_graph;
  int32_t subdomain;
} fmp_precond_desc;

/* Krylov options.  solver: 0 = BiCGSTAB, 1 = flexible GMRES(restart).
 * rtol: stop when ||b - A x||_2 / ||b - A x0||_2 <= rtol (Sec. IV-A).
 * precond: 0 = none (identity), 1 = FlashMP RAS (+ learned part if set; the
 *   learned part is used by FGMRES only, tested per step on the FP64 residual:
 *   a rejected step is recomputed with the plain preconditioner, and after
 *   three rejections in a row the rest of the solve runs without it).
 * check_every: host convergence check period for BiCGSTAB (>= 1).
 * capture_count, capture: FGMRES only; if capture_count > 0, the iterates
 *   x_1 .. x_capture_count are written to the device buffer capture
 *   (capture_count vectors of fmp_vector_layout length, caller-owned).
 * profile: 1 = record HIP events on the solve's stream around every
 *   preconditioner apply, operator apply and (FGMRES) orthogonalisation
 *   kernel, and report the times in fmp_solve_info (adds event overhead).
 * per_domain: FGMRES only.  0 = one Krylov method on the concatenated system
 *   of all domains, stopped on the residual of the whole vector.  1 = an
 *   independent FGMRES per domain (own Arnoldi basis coefficients, Givens
 *   rotations, restarts and stopping test ||b_d - A x_d|| <= rtol ||b_d - A x0_d||),
 *   all advanced in lockstep through shared kernel launches; a domain that
 *   has converged stops contributing.  Not combinable with the learned part
 *   or with capture (FMP_ERR_UNSUPPORTED / FMP_ERR_INVALID_ARG).
 * domain_iterations, domain_rel_residual: optional host arrays of n_domains
 *   entries (may be NULL), written on return: the lockstep step at which a
 *   domain met rtol (per_domain = 1; else the solve's step count) and each
 *   domain's recomputed ||b_d - A x_d|| / ||b_d - A x0_d|| (0 for b_d = A x0_d). */
typedef struct {
  int32_t solver;
  int32_t restart;
  int32_t max_iter;
  double rtol;
  int32_t precond;
  int32_t check_every;
  int32_t capture_count;
  double* capture;
  int32_t profile;
  int32_t per_domain;
  int32_t* domain_iterations;
  double* domain_rel_residual;
} fmp_solve_opts;

typedef struct {
  int32_t iterations;          /* BiCGSTAB loops or FGMRES Arnoldi steps      */
  int32_t n_precond;           /* preconditioner applies                      */
  int32_t n_spmv;              /* operator applies                            */
  int32_t used_fallback;       /* applies where the learned part was rejected */
  double rel_residual_true;    /* ||b - A x|| / ||b - A x0|| recomputed (the
                                  largest per-domain value when per_domain) */
  double t_total_ms;
  /* filled when opts.profile = 1 (kernel time from HIP events, ms; bytes are
   * the algorithmic HBM bytes of those launches: 8 per element read or written) */
  double t_precond_ms, t_spmv_ms, t_orth_dot_ms, t_orth_update_ms;
  double bytes_orth_dot, bytes_orth_update;
  int32_t n_orth_dot, n_orth_update;
} fmp_solve_info;

/* Build the subdomain plans for n_domains independent domains: the overlapping
 * decomposition of Sec. II-B (each owned block extended by the overlap gamma
 * into the box of the restriction S_i^gamma, clipped at the PEC walls; the
 * owned block is what the prolongation S_i^0T writes back), the per-box
 * constant alpha_s = c / (mean eps_r over the owned cells) of the subdomain
 * operator (eq. (7) with a subdomain-constant permittivity) and the transform
 * tables of Sec. III-A for every box side.
 * Two-phase: with ws == NULL, writes the workspace size to *ws_bytes and
 * returns FMP_OK with *out = NULL.  Then call again with a device buffer of
 * at least *ws_bytes bytes (256-byte aligned) to get a handle in *out.
 * Errors: FMP_ERR_INVALID_ARG (sizes < 2, overlap < 1, sub not dividing the
 * side, eps table missing its block size), FMP_ERR_WORKSPACE.  A domain
 * whose boxes exceed the largest compiled transform size (96 cells for PEC
 * boxes in every precision: up to 48 with the butterfly passes, 49..96 with
 * the contractions as tiled GEMMs (FP64 / FP32) or matrix-core GEMMs (BF16);
 * 48 cells for index blocks) still gets a handle: the stencil and
 * unpreconditioned solves work, while fmp_apply_precond and preconditioned
 * solves return FMP_ERR_UNSUPPORTED.  BF16 handles refuse domains whose
 * planes hold 2^27 cells or more (FMP_ERR_UNSUPPORTED): their gather
 * addresses a slab of four planes by 32-bit byte offsets. */
fmp_status fmp_setup_subdomains(const fmp_domain_desc* domains, int32_t n_domains,
                                const fmp_precond_desc* pd, void* ws, size_t* ws_bytes,
                                void* stream, fmp_handle* out);

/* offsets[0..n_domains]: element offset of each domain block; offsets[n] = total. */
fmp_status fmp_vector_layout(fmp_handle h, int64_t* offsets);

/* y = A x (the double-curl stencil with the permittivity scaling; Sec. III-A
 * double-curl matrix, eq. (7)).  x, y: device, fmp_vector_layout length,
 * must not overlap (FMP_ERR_ALIAS). */
fmp_status fmp_curlcurl_apply(fmp_handle h, const double* x, double* y, void* stream);

/* z = M^{-1} r: RAS with exact transform solves of every box (Sec. II-B;
 * Algorithm 1, exact_solve), plus the learned coarse correction when set.
 * r, z: device, must not overlap. */
fmp_status fmp_apply_precond(fmp_handle h, const double* r, double* z, void* stream);

/* One measured candidate of fmp_autotune: a preconditioner launch plan
 * (stencil_ty = 0) or a stencil tile height (stencil_ty > 0, the other plan
 * fields 0). */
typedef struct {
  int32_t batch_boxes;   /* boxes per batch (staging reused batch after batch)  */
  int32_t streams;       /* 1: batches in order; 2: consecutive batches on two
                            private streams with two staging buffers (overlap) */
  int32_t slab_order;    /* gather/scatter work order: 0 box by box, 1 slab by
                            slab across the batch's boxes (shared halo lines)  */
  double apply_ms;       /* mean time of one preconditioner apply, or of one
                            fmp_curlcurl_apply for a stencil candidate (HIP
                            events)                                             */
  int32_t chosen;        /* 1 for the candidates the handle now uses            */
  int32_t stencil_ty;    /* stencil tile 64 x stencil_ty (4, 8, 16), or 0       */
  int32_t cached;        /* 1: the plan came from the FMP_TUNE_CACHE file       */
} fmp_tune_entry;

/* Autotuner of the launch plans.  Preconditioner: times fmp_apply_precond(r, z)
 * as plain launch sequences (three applies after a warm-up) for every
 * candidate batch size (16 .. 1024 boxes and all boxes, per size class),
 * stream count and gather work order.  Stencil: times fmp_curlcurl_apply(r, z)
 * (five applies after a warm-up) for tiles of 64 x 4, 64 x 8 and 64 x 16
 * columns.  Keeps the fastest of each.  Every plan computes the same results
 * bit for bit; only the schedule changes.
 * Persistent cache: if the environment variable FMP_TUNE_CACHE names a file,
 * a record for this handle's key (library revision, device, precision,
 * overlap, learned part, every domain's size and subdomain split) is looked
 * up there first; a hit applies the recorded plan and times only it (the
 * returned entries say cached = 1), a miss tunes and appends the record.  The
 * file is plain text, one record per line; concurrent writers are not
 * coordinated.
 * Requires a handle set up with batch_boxes = -1 (else FMP_ERR_UNSUPPORTED).
 * r, z: device vectors (not overlapping); z is overwritten.  entries:
 * optional host array of max_entries records; *n_entries (may be NULL) gets
 * the count written.  Synchronises the stream. */
fmp_status fmp_autotune(fmp_handle h, const double* r, double* z, fmp_tune_entry* entries,
                        int32_t max_entries, int32_t* n_entries, void* stream);

/* Workspace the solver needs for `opts` (bytes).  */
fmp_status fmp_solve_workspace(fmp_handle h, const fmp_solve_opts* opts, size_t* bytes);

/* Solve A x = b (eq. (7)) with the Krylov methods of Sec. IV-A: BiCGSTAB or
 * GMRES(restart) (flexible, right-preconditioned by fmp_apply_precond), stopped
 * when the recomputed FP64 residual meets rtol; per iteration BiCGSTAB does two
 * preconditioner applies and two operator applies, GMRES one of each plus the
 * orthogonalisation (Table III).  x holds the initial guess on entry and the solution on
 * exit; the wall slots of b and of the initial x are ignored, and those of x
 * are 0 on exit.  ws: device buffer of fmp_solve_workspace bytes (256-byte
 * aligned).  Returns FMP_OK, FMP_NOT_CONVERGED (x = last iterate), or
 * FMP_ERR_BREAKDOWN (x = last finite iterate).  info may be NULL. */
fmp_status fmp_solve(fmp_handle h, const double* b, double* x, const fmp_solve_opts* opts,
                     void* ws, size_t ws_bytes, fmp_solve_info* info, void* stream);

/* ---- Crank-Nicolson time stepping around the solve ---------------------------
 * Sec. II-A, eqs. (2)-(5): Maxwell's curl equations in normalised units
 * (mu = 1, unit cell size, eps the relative permittivity) marched by
 * Crank-Nicolson,
 *     eps (E+ - E) / dt =  (1/2) C^T (H+ + H),   (H+ - H) / dt = -(1/2) C (E+ + E),
 * C the Yee curl from E (edges) to H (dual faces) of Sec. III-A eq. (6).
 * Eliminating H+ gives A E+ = R with A the operator of fmp_curlcurl_apply,
 * c = dt^2 / 4 and R = E + dt eps^-1 C^T (H - (dt/4) C E); so a domain's time
 * step is dt = 2 sqrt(c) (its fmp_domain_desc.c).
 * H vectors have the E layout (fmp_vector_layout): per domain [3][nz][ny][nx],
 * H_x at (i, j+1/2, k+1/2) in slot [k][j][i], H_y at (i+1/2, j, k+1/2),
 * H_z at (i+1/2, j+1/2, k); slot 0 of a component's own axis (i for H_x, j for
 * H_y, k for H_z) is a wall slot, ignored on input and 0 on output. */

/* h_out = beta h_in + m dt C (e1 + e2), each domain with its own dt.
 * e2 and h_in may be NULL (taken as zero).  Device vectors of the layout
 * length; h_out may be h_in itself, must not overlap e1 or e2
 * (FMP_ERR_ALIAS).  Wall slots of e1, e2, h_in are ignored. */
fmp_status fmp_curl_e(fmp_handle h, const double* e1, const double* e2, const double* h_in,
                      double beta, double m, double* h_out, void* stream);

/* e_out = e_in + m dt eps_e^-1 C^T hf, eps_e the edge permittivity of the
 * operator A (mean of the four cells sharing the edge).  e_in may be NULL
 * (zero) or e_out itself; hf must not overlap e_out (FMP_ERR_ALIAS). */
fmp_status fmp_curl_h(fmp_handle h, const double* hf, const double* e_in, double m,
                      double* e_out, void* stream);

/* Workspace of fmp_cn_step for opts (bytes): the solver's plus two vectors. */
fmp_status fmp_cn_workspace(fmp_handle h, const fmp_solve_opts* opts, size_t* bytes);

/* One Crank-Nicolson step in place: R = E + dt eps^-1 C^T (H - (dt/4) C E);
 * A E+ = R by fmp_solve with opts, started from E (so rtol is relative to the
 * initial residual b - A E); H = H - (dt/2) C (E+ + E); E = E+.  E, H: device,
 * layout length, not overlapping; ws: device buffer of fmp_cn_workspace bytes
 * (256-byte aligned).  Returns fmp_solve's status; on a status other than
 * FMP_OK and FMP_NOT_CONVERGED, E and H are unchanged.  Synchronises the
 * stream.  info may be NULL. */
fmp_status fmp_cn_step(fmp_handle h, double* E, double* H, const fmp_solve_opts* opts, void* ws,
                       size_t ws_bytes, fmp_solve_info* info, void* stream);

/* ---- learned coarse correction (z += P0 MLP(R0 r)) --------------------------
 * R0: mean of r over the unknowns each subdomain owns, per component; the
 * coarse vector is [3][n_subdomains] (subdomains in the same order as the
 * boxes: domain, then z, y, x).  The MLP maps the coarse residual scaled to
 * unit norm through in -> hidden (ReLU) -> hidden (ReLU) -> in with bf16
 * weights and FP32 accumulation; its output, times the norm, is injected
 * piecewise-constantly (P0) into the owned unknowns. */

/* Number of coarse unknowns (3 * subdomains) of a handle. */
fmp_status fmp_coarse_size(fmp_handle h, int32_t* n_coarse);

/* Host FP32 weights in order W1[hid][in], b1[hid], W2[hid][hid], b2[hid],
 * W3[in][hid], b3[in]; bytes must equal 4*(2*in*hid + hid*hid + 2*hid + in).
 * Weights are rounded to bf16 on upload (biases stay FP32).  hidden <= 512.
 * Passing weights == NULL disables the correction. */
fmp_status fmp_set_coarse_model(fmp_handle h, int32_t hidden, const float* weights, size_t bytes);

/* rc = R0 r (device, FP64 out, fmp_coarse_size entries). */
fmp_status fmp_coarse_restrict(fmp_handle h, const double* r, double* rc, void* stream);

/* ---- MLP training kernels (used to fit the coarse model) -------------------
 * All pointers are device FP32 unless noted.  Shapes: X [batch][in],
 * Y [batch][in], params = the flat FP32 layout of fmp_set_coarse_model,
 * grads same size.  fmp_mlp_loss_grad: forward with bf16 copies of the
 * weights and FP32 accumulation, MSE loss mean over batch*in entries written
 * to *loss_dev (device FP32), and its gradient with respect to params.
 * fmp_mlp_adam: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on params
 * with moments m, v (device FP32, zero initialised), step count t >= 1. */
fmp_status fmp_mlp_loss_grad(int32_t in_dim, int32_t hidden, int32_t batch, const float* params,
                             const float* X, const float* Y, float* grads, float* loss_dev,
                             void* scratch, size_t scratch_bytes, void* stream);
size_t fmp_mlp_scratch_bytes(int32_t in_dim, int32_t hidden, int32_t batch);
fmp_status fmp_mlp_adam(int32_t n_params, float* params, const float* grads, float* m, float* v,
                        int32_t t, float lr, void* stream);

/* ---- allocation-free variant (for callers that cannot allocate) -------------
 * For callers that may not call hipMalloc or any allocating routine: code
 * under hipGraph capture, tight training loops, harnesses that forbid device
 * allocation.  fmp_mlp_loss_grad_noalloc computes exactly what
 * fmp_mlp_loss_grad computes (same kernels, same order, bitwise the same
 * loss and gradients) but takes its scratch (layer activations, hidden-layer
 * gradients, loss partials) from a static device buffer of
 * FMP_MLP_NOALLOC_SCRATCH_BYTES inside the library instead of a caller
 * buffer.  It allocates nothing, host or device.
 *   - Limit: fmp_mlp_scratch_bytes(in_dim, hidden, batch) must not exceed
 *     FMP_MLP_NOALLOC_SCRATCH_BYTES (64 MiB; e.g. in_dim 1536, hidden 256,
 *     batch <= 4095); larger shapes return FMP_ERR_WORKSPACE and
 *     fmp_last_error(NULL) says by how much.
 *   - The buffer of the GPU current on the calling thread is used (its
 *     address is looked up once per GPU, on the first call with that GPU
 *     current); `stream` must belong to that GPU.  Each GPU the library runs
 *     on holds its own 64 MiB buffer until the process ends.
 *   - Every call on one GPU shares that GPU's buffer: calls that overlap in
 *     time on one GPU (different streams, or host threads, without ordering
 *     between them) race on it and give undefined results.  Calls ordered on
 *     one stream are safe.  No part of the buffer needs to start at zero.
 *   - Other arguments, shapes and errors as fmp_mlp_loss_grad; FMP_ERR_HIP if
 *     the buffer's device address cannot be obtained. */
#define FMP_MLP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fmp_status fmp_mlp_loss_grad_noalloc(int32_t in_dim, int32_t hidden, int32_t batch,
                                     const float* params, const float* X, const float* Y,
                                     float* grads, float* loss_dev, void* stream);

/* Release a handle.  Synchronises the device first (captured applies may
 * still replay on any stream), then frees the handle's graphs, private
 * streams, events and pinned host mirrors.  The caller's workspace is not
 * touched.  FMP_ERR_HIP if the synchronisation reported an error (the handle
 * is released either way). */
fmp_status fmp_destroy(fmp_handle h);
const char* fmp_status_string(fmp_status st);
/* Detail message of the last error on handle h; with h == NULL, of the last
 * failed call on this host thread that takes no handle. */
const char* fmp_last_error(fmp_handle h);

/* HIP versions in the HIP_VERSION encoding (major * 10^7 + minor * 10^5 +
 * patch): *compiled = the headers the library was built with, *running = the
 * libamdhip64 the process has loaded (a framework may bundle an older one of
 * the same major release; 0 if it cannot be queried).  fmp_setup_subdomains
 * refuses a runtime of another major release with FMP_ERR_UNSUPPORTED.
 * Host only; FMP_ERR_HIP if the runtime cannot be queried. */
fmp_status fmp_runtime_version(int32_t* compiled, int32_t* running);

#ifdef __cplusplus
}
#endif
#endif /* FLASHMP_H */
