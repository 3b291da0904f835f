/*
 * ds3.h — C ABI of the dense Sim(3) back-end for AMD MI355X (gfx950).
 *
 * The library implements the data-parallel back-end path of CoMo3R-SLAM (collaborative monocular dense
 * SLAM with learned 3D priors): bidirectional projective matching of dense pointmaps between keyframe
 * pairs (Sec. III-A "Learned geometry", Sec. III-B), gauge synchronisation of map components
 * (Sec. III-C, eqs. 3-4), and Gauss-Newton/IRLS refinement of the unified Sim(3) keyframe graph
 * (Sec. III-D, eqs. 1, 5, 6, 7), plus the gradient of the graph cost (eq. 5) with respect to pointmaps,
 * confidences and poses.
 *
 * Conventions shared by every call
 *   - Pointers marked (device) are HIP device pointers owned by the caller; pointers marked (host) are
 *     host memory read during the call. The library never frees caller memory.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*, NULL = default stream) unless
 *     the description says the call synchronises. Results are valid after the stream completes.
 *   - Return value: DS3_OK (0) or a negative DS3_E* code. ds3_status_string() gives a description of
 *     the last error of the calling thread. No C++ exception crosses this boundary.
 *   - Numerical failure of the pose solve is NOT an error: following the text after eq. (7) it yields
 *     a zero update and status -1 (see ds3_sim3_gn_step).
 *   - Pose layout (float64, 8 per keyframe): [tx, ty, tz, qx, qy, qz, qw, s], T_WC = [[sR, t], [0, 1]]
 *     with R from the unit quaternion and s > 0 (Sec. III-A, "Ray-range tracking").
 *   - Tangent layout (float64, 7 per keyframe): tau = (v, omega, zeta), T <- Exp(tau) T (Sec. III-D).
 *   - Pixel grid: row-major, pixel (u, v) at index v*W + u, u the column.
 *   - Keyframe data lives in an "xyzc arena": per pixel x, y, z of the canonical pointmap (the
 *     keyframe's points in its own camera frame) and its confidence c, packed as 4 x float32 (16 B,
 *     DS3_F32) or 4 x bfloat16 (8 B, DS3_BF16, round-to-nearest-even). Arenas are 16 B aligned.
 */
#ifndef DS3_H
#define DS3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DS3_OK 0
#define DS3_EINVAL (-1)   /* null pointer, bad size, misaligned arena, index out of range */
#define DS3_ENOTSUP (-2)  /* unsupported dtype or device architecture */
#define DS3_EHIP (-3)     /* HIP runtime error (detail in ds3_status_string) */
#define DS3_ENOSPACE (-4) /* workspace smaller than the size the *_workspace_bytes call returned */
#define DS3_EDEGENERATE (-5) /* degenerate input with no unique answer (collinear correspondences) */

typedef enum { DS3_F32 = 0, DS3_BF16 = 1 } ds3_dtype;

/* One keyframe image inside an xyzc arena: H x W pixels starting at pixel px_offset. */
typedef struct {
  int32_t H, W;
  int64_t px_offset;
} ds3_image;

/* One graph edge (i, j) of E_global (eq. 5): its matches are H_j*W_j int32 entries at idx_offset of an
 * idx arena; entry n is the pixel m of keyframe i matched to pixel n of keyframe j, or -1. */
typedef struct {
  int32_t i, j;
  int64_t idx_offset;
} ds3_edge;

/* Matching constants. nu_min is the paper's admission gate (Sec. III-B, 0.1). The remaining values are
 * readings where the paper is silent: Levenberg-Marquardt on the bilinear ray interpolant (max_iters
 * trial steps, damping lambda0, floor lambda_min, stop after a trial step (accepted or not) below
 * step_tol_px in a non-singular system),
 * validity = no hole, final angular residual <= ang_tol_px * min(|ds/du|, |ds/dv|), and
 * | |x| - |X_ref[idx]| | <= range_rel_tol * |X_ref[idx]|; mutual check within a Chebyshev radius;
 * q_min the confidence sqrt(C_i C_j) needed to count towards nu.
 * Defaults: 10, 1e-4, 1e-9, 1e-4, 0.5, 0.10, 1, 1.5, 0.1. */
typedef struct {
  int32_t max_iters;
  double lambda0, lambda_min, step_tol_px, ang_tol_px, range_rel_tol;
  int32_t mutual_radius_px;
  double q_min, nu_min;
} ds3_match_params;

/* Graph-step constants: sigma_r = 0.003, sigma_d = 10, Huber kappa = 1.345 (Sec. IV-A); eq. (7) damping
 * lambda (0 for the back-end) and the epsilon ladder eps_r = eps0 * eps_mult^r, r < max_attempts
 * (1e-6, 100, 6; text after eq. 7).
 * Calibrated mode (Sec. IV-C, "Calibration"): K != NULL (host, n_kf x 4 float64: fx, fy, cx, cy per
 * keyframe, in the keyframe table's order) replaces the ray-range residual of eq. (1) by pixel
 * reprojection and log-depth on the pointmaps constrained to the calibrated rays: for a match (m, n) of
 * edge (i, j), Xcal_j[n] = z_j[n] K_j^-1 (u_n, v_n, 1) with z = the stored point's third coordinate,
 * x = T_ij Xcal_j[n], r = (fx_i x0/x2 + cx_i - u_m, fy_i x1/x2 + cy_i - v_m, ln x2 - ln z_i[m]), whitened by
 * sqrt(q)/sigma_pix and sqrt(q)/sigma_logz (q = sqrt(C_i C_j)), the same Huber kernel; matches with a
 * hole, z_j[n] or z_i[m] <= 1e-9, x2 <= 1e-9, or a reprojection off keyframe i's image (outside
 * [-0.5, W_i - 0.5) x [-0.5, H_i - 0.5)) are skipped. The paper prints no constants for this mode:
 * sigma_pix = 1 px and sigma_logz = 0.1 are readings. Supported by ds3_gn_linearize, ds3_sim3_gn_step and
 * the batched plan; the cost, adjoint and tracker calls return DS3_ENOTSUP when K is set. */
typedef struct {
  double sigma_ray, sigma_dist, huber_k, lambda, eps0, eps_mult;
  int32_t max_attempts;
  const double* K;
  double sigma_pix, sigma_logz;
} ds3_gn_params;

void ds3_default_match_params(ds3_match_params* p);
void ds3_default_gn_params(ds3_gn_params* p);
const char* ds3_status_string(int code);
int ds3_version(void);

/* ---------------------------------------------------------------------------------------------------
 * Keyframe layout (ray operator input, Sec. III-A)
 * ------------------------------------------------------------------------------------------------- */

/* Pack n_px pixels of xyz (device, float32, 3 per px) and conf (device, float32) into an xyzc arena
 * (device, 16 B per px for DS3_F32, 8 B for DS3_BF16 with round-to-nearest-even; NaN stays NaN). */
int ds3_pack_xyzc(const float* xyz, const float* conf, int64_t n_px, ds3_dtype dtype, void* xyzc_out,
                  void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Projective matching (Sec. III-A "Learned geometry": p* = argmin_p |psi([X_ref]_p) - psi(x)|^2) and
 * bidirectional verification (Sec. III-B)
 * ------------------------------------------------------------------------------------------------- */

/* Workspace bytes for ds3_match (one direction) and ds3_match_bidir. */
size_t ds3_match_workspace_bytes(int32_t H_ref, int32_t W_ref);
size_t ds3_match_bidir_workspace_bytes(int32_t H_i, int32_t W_i, int32_t H_j, int32_t W_j);

/* One direction. ref_xyzc: the reference keyframe's canonical pointmap (device arena, image `ref`).
 * qry_xyzc: the other view's points expressed in the reference camera (device arena, image `qry`), its
 * confidence in c. For every query pixel n: idx_out[n] (device, int32, H_q*W_q) = v*W_ref + u of
 * round(p*) (ties up), or -1 when the query is a hole, a bilinear sample touched a hole, or a validity
 * test failed. Optional diagnostics (device, may be NULL): p_out (2 float per query, the continuous
 * optimum), iters_out (int32, LM trial steps). Needs H_ref, W_ref >= 2. */
int ds3_match(const void* ref_xyzc, ds3_image ref, const void* qry_xyzc, ds3_image qry, ds3_dtype dtype,
              const ds3_match_params* params, int32_t* idx_out, float* p_out, int32_t* iters_out,
              void* workspace, size_t ws_bytes, void* stream);

/* Both decoded directions of a candidate pair, the mutual check and the nu gate.
 *   X_ii: canonical pointmap of i (image img_i), X_ji: j's points in camera i (image img_j geometry),
 *   X_jj: canonical pointmap of j, X_ij: i's points in camera j (img_i geometry); all device arenas
 *   with confidences in c.
 * Outputs (device): idx_j2i (int32 H_j*W_j; the match of pixel n of j in i, -1 unless mutually valid),
 *   valid_j (uint8 H_j*W_j), nu (float32 [nu_i, nu_j]: fraction of pixels of i resp. j with a mutually
 *   valid match of confidence sqrt(C_i C_j) >= q_min), admit (int32: min(nu) >= nu_min). */
int ds3_match_bidir(const void* X_ii, const void* X_ji, const void* X_jj, const void* X_ij,
                    ds3_image img_i, ds3_image img_j, ds3_dtype dtype, const ds3_match_params* params,
                    int32_t* idx_j2i, uint8_t* valid_j, float* nu, int32_t* admit, void* workspace,
                    size_t ws_bytes, void* stream);

/* Kernel timer: two HIP events (timing enabled, created on the current device) that a library call
 * records on its stream immediately before and after one kernel launch, so that the caller can read that
 * kernel's duration without a profiler. Calls that would record it inside a stream capture fail with
 * DS3_ENOTSUP. ds3_timer_elapsed_ms waits for the second event and returns the time between the last
 * recorded pair in *ms (host); DS3_EINVAL if nothing was recorded yet. */
typedef struct ds3_timer ds3_timer;
int ds3_timer_create(ds3_timer** out);
int ds3_timer_elapsed_ms(ds3_timer* timer, float* ms);
int ds3_timer_destroy(ds3_timer* timer);

/* Batched bidirectional matching of many edges in few launches.
 *   kf_arena (device) + kf (host, n_kf images): canonical pointmaps.
 *   cross_arena (device): per edge e two cross-view pointmaps, X^j_i (H_j*W_j px) at cross_off[2e] and
 *   X^i_j (H_i*W_i px) at cross_off[2e+1] (host int64 pixel offsets).
 *   edges (host): (i, j, idx_offset) per edge; outputs written at idx_offset of idx_arena (int32) and
 *   valid_arena (uint8); nu (device float32, 2 per edge), admit (device int32, 1 per edge);
 *   lm_steps (device uint64, may be NULL) receives the total number of LM trial steps taken;
 *   match_timer (may be NULL) is recorded around the one launch that runs every LM query.
 * Workspace from ds3_match_batch_workspace_bytes. */
size_t ds3_match_batch_workspace_bytes(int32_t n_kf, const ds3_image* kf, int32_t n_edges,
                                       const ds3_edge* edges);
int ds3_match_batch(const void* kf_arena, const ds3_image* kf, int32_t n_kf, const void* cross_arena,
                    const int64_t* cross_off, const ds3_edge* edges, int32_t n_edges, ds3_dtype dtype,
                    const ds3_match_params* params, int32_t* idx_arena, uint8_t* valid_arena, float* nu,
                    int32_t* admit, uint64_t* lm_steps, ds3_timer* match_timer, void* workspace,
                    size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Gauge synchronisation (Sec. III-C)
 * ------------------------------------------------------------------------------------------------- */

/* Closed-form similarity of eq. (4) between the matches of one admitted edge lifted to world frames:
 * x = T_i X_i[m], y = T_j X_j[n] over valid_j. ref_is_i = 1 aligns j's component onto i's (T* maps y to
 * x), 0 the reverse. With fewer than nc_min correspondences, or a rank < 2 cross-covariance, T* is the
 * endpoint transform T_ref T_mov^-1. Outputs (device): T_out (8 float64), used_umeyama (int32). */
int ds3_gauge_align(const void* X_i, ds3_image img_i, const void* X_j, ds3_image img_j, ds3_dtype dtype,
                    const int32_t* idx_j2i, const uint8_t* valid_j, const double* poses, int32_t i,
                    int32_t j, int32_t ref_is_i, int32_t nc_min, double* T_out, int32_t* used_umeyama,
                    void* workspace, size_t ws_bytes, void* stream);
/* The closed form of eq. (4) on the host, float64: the similarity T* = (s, R, t) minimising
 * sum_l |x_l - (s R y_l + t)|^2 over n correspondences x, y (host, n x 3 float64 each, row l = point l),
 * written as a pose (T_out, host, 8 float64: T* maps y onto x). With centroids xb, yb and
 * A = (1/n) sum (x - xb)(y - yb)^T = U Lambda V^T: R = U S V^T with S = diag(1, 1, det(U V^T)),
 * s = tr(S Lambda) / ((1/n) sum |y - yb|^2), t = xb - s R yb (the same solve the device gauge alignment
 * uses). Returns DS3_EINVAL for null pointers, n < 1 or non-finite input, and DS3_EDEGENERATE (T_out
 * untouched) when rank(A) < 2 (collinear points: the rotation about their line is free) or y has no
 * spread. No GPU call. */
int ds3_umeyama(const double* x, const double* y, int64_t n, double* T_out);

/* Workspace bytes of ds3_gauge_align and ds3_gauge_sync for a graph of n_kf keyframes. */
size_t ds3_gauge_workspace_bytes(int32_t n_kf);

/* Left-multiply T (device, 8 float64) onto every pose k (device, n_kf x 8) with mask[k] != 0 (device
 * uint8): re-gauges a map component while keeping its internal relative poses. */
int ds3_apply_gauge(double* poses, int32_t n_kf, const uint8_t* mask, const double* T, void* stream);

/* The component tracker of Sec. III-C over a whole graph: walks the edges in order; every admitted
 * edge (admit, device int32 per edge) between keyframes of different agents (agent_of_kf, host) whose
 * agents are still in different components aligns the moving component onto the reference (the one
 * holding agent 0, else the one with the smaller smallest agent id) with ds3_gauge_align and
 * ds3_apply_gauge. Synchronises the stream once to read the admit flags. n_links_out (host) receives
 * the number of merges. */
int ds3_gauge_sync(double* poses, int32_t n_kf, const int32_t* agent_of_kf, const void* kf_arena,
                   const ds3_image* kf, ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges,
                   const int32_t* idx_arena, const uint8_t* valid_arena, const int32_t* admit,
                   int32_t nc_min, int32_t* n_links_out, void* workspace, size_t ws_bytes,
                   void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Sim(3) (Sec. III-A pose model, Sec. III-D left perturbation); float64 on the device
 * ------------------------------------------------------------------------------------------------- */
int ds3_sim3_exp(const double* tau, double* poses_out, int32_t n, void* stream);
int ds3_sim3_log(const double* poses, double* tau_out, int32_t n, void* stream);
/* poses[k] <- Exp(tau[k]) poses[k] for every k with fixed == NULL or fixed[k] == 0 (device arrays). */
int ds3_sim3_update(double* poses, const double* tau, const uint8_t* fixed, int32_t n, void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Graph step (eqs. 1, 5, 6, 7)
 * ------------------------------------------------------------------------------------------------- */

/* Workspace bytes of ds3_gn_linearize / ds3_sim3_gn_step / ds3_gn_cost / ds3_gn_cost_adjoint for a
 * graph with n_kf keyframes and these edges (host), at this dtype. */
size_t ds3_gn_workspace_bytes(int32_t n_kf, const ds3_image* kf, int32_t n_edges, const ds3_edge* edges,
                              ds3_dtype dtype);

/* Assemble the normal equations of eq. (7) at `poses` (device, n_kf x 8):
 * H (device, (7 n_kf)^2 float64, row-major, full symmetric) and g (device, 7 n_kf float64) summed over
 * every valid match of every edge (eq. 5), with the rows and columns of each anchor keyframe (host list)
 * replaced by identity and its g by 0; cost_out (device float64) = E_global at `poses`; count_out
 * (device int64, may be NULL) = matches used. Pixels with idx = -1, non-finite or zero-range points and
 * non-finite confidences are skipped. Plain form: one launch per edge. */
int ds3_gn_linearize(const double* poses, int32_t n_kf, const ds3_image* kf, const void* xyzc_arena,
                     ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges, const int32_t* idx_arena,
                     const ds3_gn_params* params, const int32_t* anchors, int32_t n_anchors, double* H,
                     double* g, double* cost_out, int64_t* count_out, void* workspace, size_t ws_bytes,
                     void* stream);

/* One Gauss-Newton/IRLS step of eq. (5) via eq. (7) (plain form: one residual launch per edge, no
 * graph): assemble as ds3_gn_linearize, solve (H + lambda diag H + eps_r I) tau = -g with the epsilon
 * ladder, update poses (device, in/out) by T <- Exp(tau) T except anchors. cost_out (device float64) =
 * E at the input poses; status_out (device int32) = ladder attempt used, -1 for a zero update after
 * max_attempts failures. tau_out (device, 7 n_kf float64) may be NULL. */
int ds3_sim3_gn_step(double* poses, int32_t n_kf, const ds3_image* kf, const void* xyzc_arena,
                     ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges, const int32_t* idx_arena,
                     const ds3_gn_params* params, const int32_t* anchors, int32_t n_anchors,
                     double* cost_out, int32_t* status_out, double* tau_out, void* workspace,
                     size_t ws_bytes, void* stream);

/* Solve (H + lambda diag(H) + eps_r I) tau = -g for a symmetric n x n H (device, row-major, float64;
 * only the lower triangle is read; 1 <= n <= 8192, else DS3_EINVAL) with eps_r = eps0 * mult^r,
 * r = 0 .. attempts-1 (attempts <= 16); tau (device, n) = 0 and status (device int32) = -1 when every
 * factorisation fails, else status = r. Workspace from ds3_chol_workspace_bytes(n). */
size_t ds3_chol_workspace_bytes(int32_t n);
int ds3_chol_ladder_solve(const double* H, const double* g, int32_t n, double lambda, double eps0,
                          double mult, int32_t attempts, double* tau, int32_t* status, void* workspace,
                          size_t ws_bytes, void* stream);

/* Block-sparse form of ds3_chol_ladder_solve for the fixed 7x7-block pattern of a pose graph (eq. (7) and
 * the epsilon ladder after it): H couples keyframes a and b only for the listed pairs.
 * ds3_spchol_analyse (host only, no device use): symbolic analysis of the pattern of n_kf keyframes
 * (1 <= n_kf <= 1170) and the n_pairs pairs pair_ij[2p], pair_ij[2p+1] (host; each in 0 .. n_kf-1,
 * a != b, repeats allowed; DS3_EINVAL otherwise): a minimum-degree elimination order (ties: lowest id),
 * the filled block pattern of the Cholesky factor and its elimination tree. Writes the elimination
 * order by tree level (perm[c] = keyframe of factor column c; host, n_kf int32; may be NULL), each
 * keyframe's tree level (level[k]; host, n_kf; may be NULL) and info (host, 6 int64): n_kf, blocks of
 * the factor (diagonal ones included), fill blocks (not in the pattern), levels, block products of the
 * factorisation, int32 words of the index tables.
 * ds3_spchol_create: the same analysis, then device copies of the tables and the factor's storage
 * (the object owns them; synchronises). DS3_ENOSPACE for more than 512 keyframes or index tables above
 * 28672 words (the solve keeps both in LDS); the dense solver takes such patterns.
 * ds3_spchol_solve: solves (H + lambda diag(H) + eps_r I) tau = -g with eps_r = eps0 * mult^r, r = 0 ..
 * attempts-1 (1 <= attempts <= 16), on `stream`, in one launch and without host synchronisation. H is
 * the symmetric (7 n_kf)^2 float64 matrix (device, row-major); only the lower triangle of its pattern
 * blocks (the diagonal blocks and the listed pairs) is read and every other block counts as zero. g, tau:
 * device, 7 n_kf float64; status (device int32) = the attempt used, or -1 with tau = 0 when every
 * factorisation meets a pivot that is not positive and finite. Calls on one object must not overlap (they
 * share its factor storage). The solve runs in one workgroup (level after level of the elimination tree;
 * a small gather kernel over the device comes first), so one compute unit's memory pipeline bounds it:
 * it does less arithmetic than the dense solver but is not faster on pose graphs of a few hundred
 * keyframes, and the plans use it only when asked (ds3_plan_opts.solver = 2). */
typedef struct ds3_spchol ds3_spchol;
int ds3_spchol_analyse(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, int32_t* perm, int32_t* level,
                       int64_t* info);
int ds3_spchol_create(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, ds3_spchol** out);
int ds3_spchol_info(const ds3_spchol* S, int64_t* info);
int ds3_spchol_solve(ds3_spchol* S, const double* H, const double* g, double lambda, double eps0, double mult,
                     int32_t attempts, double* tau, int32_t* status, void* stream);
void ds3_spchol_destroy(ds3_spchol* S);

/* Tile-sparse form of ds3_chol_ladder_solve for the same keyframe-pair pattern (eq. (7) and the epsilon
 * ladder after it). The dense solver's float64 32x32 tiles, laid out so that the pose graph's independent
 * parts fall into different tiles: an elimination order of the keyframe graph (minimum degree, or nested
 * dissection cut at the balanced breadth-first level or at the smallest separator one level around it), a
 * postorder of its elimination tree in which sibling subtrees of at least `thr` keyframes (all but the
 * largest child of a node) start and end on tile boundaries (padding rows are identity rows), the symbolic
 * tile factorisation of that layout and its tile elimination tree; the order and threshold with the fewest
 * tree levels, then the fewest tiles, are kept. Attempt 0 then runs one launch per tree
 * level (instead of one per 32-row panel) and a dataflow back substitution over the tree; attempts 1..
 * run in the dense solver's persistent fallback.
 * ds3_tilechol_analyse (host only, no device use): the analysis of n_kf keyframes (1 <= n_kf <= 1170)
 * and the n_pairs pairs pair_ij[2p], pair_ij[2p+1] (host; each in 0 .. n_kf-1, a != b, repeats allowed;
 * DS3_EINVAL otherwise). Writes each keyframe's first row in the tile layout (kf_row0[k]: its 7 rows are
 * kf_row0[k] .. +6; host, n_kf int32; may be NULL) and info (host, 7 int64): n_kf, tiles per side of the
 * layout, factor tiles (lower, diagonal included, fill included), tree levels, tile updates (trailing
 * tile x pivot products), padding rows, the threshold chosen (the fewest levels, then the fewest factor
 * tiles, over 2, 3, 4, 6, 9, 14, 20 and no alignment). DS3_ENOSPACE when every layout has more than 1024
 * tiles per side.
 * ds3_tilechol_create: the same analysis, then device copies of the tables and the factor's storage
 * (the object owns them: 16 KiB per factor tile; synchronises).
 * ds3_tilechol_solve: solves (H + lambda diag(H) + eps_r I) tau = -g with eps_r = eps0 * mult^r, r = 0 ..
 * attempts-1 (1 <= attempts <= 16), on `stream`, without host synchronisation. H: the symmetric
 * (7 n_kf)^2 float64 matrix (device, row-major); only the lower triangle of its pattern blocks (the
 * diagonal blocks and the listed pairs) is read and every other block counts as zero. g, tau: device,
 * 7 n_kf float64; status (device int32) = the attempt used, -1 with tau = 0 when every factorisation
 * meets a pivot that is not positive and finite, -2 when a bounded wait of the back substitution timed
 * out. workspace: caller-owned device memory of at least ds3_chol_workspace_bytes(7 n_kf) bytes (its
 * synchronisation words and the fallback's storage; DS3_ENOSPACE when workspace_bytes is smaller). Calls
 * on one object or one workspace must not overlap. */
typedef struct ds3_tilechol ds3_tilechol;
int ds3_tilechol_analyse(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, int32_t* kf_row0,
                         int64_t* info);
int ds3_tilechol_create(int32_t n_kf, int32_t n_pairs, const int32_t* pair_ij, ds3_tilechol** out);
int ds3_tilechol_info(const ds3_tilechol* S, int64_t* info);
int ds3_tilechol_solve(ds3_tilechol* S, const double* H, const double* g, double lambda, double eps0,
                       double mult, int32_t attempts, double* tau, int32_t* status, void* workspace,
                       size_t workspace_bytes, void* stream);
void ds3_tilechol_destroy(ds3_tilechol* S);

/* Batched form: one plan per graph topology (edges, keyframe images, idx offsets) over a set of matches.
 * The matches and the pointmaps stay fixed while Gauss-Newton moves the poses, so the plan holds a match
 * stream: for every edge, the two arena entries (X_j[n] and X_i[m]) and the weight (C_i C_j)^(1/4) of each
 * valid match, gathered once into contiguous records (16 B per match for DS3_BF16, 32 B for DS3_F32),
 * grouped in segments of 256 * px_per_thread pixels of keyframe j; matches with a hole, a non-finite value
 * or a negative confidence product are dropped here, as the plain form skips them. Every iteration then
 * streams those records (one block per segment, the heaviest segments first), instead of scanning the
 * idx arena and gathering X_i again. Creation uploads the topology, gathers the stream, picks the
 * segment size and the loads in flight per thread (opts->autotune: timed candidates, cached per device,
 * dtype and shape mix; synchronises) and captures one GN iteration, and eight back to back, in hipGraphs.
 * The plan owns its device buffers (the stream: up to (sum over edges of H_j*W_j, rounded up to whole
 * segments) records) and its graph; the keyframe arena, idx arena and poses stay the caller's and must
 * outlive the plan. After the caller rewrites the idx arena (a new matching pass) or the keyframe arena,
 * ds3_gn_plan_refresh must run before the next ds3_gn_plan_run: the plan reads the snapshot, not the
 * arenas. ds3_gn_plan_run replays the iteration `iters` times on `stream` with no host synchronisation
 * (eight at a time through the eight-iteration graph while at least eight remain: a replay pays a launch
 * gap of several microseconds before its first kernel),
 * writing E at each iteration's input poses to cost_per_iter (device, iters float64) and the ladder status
 * to status_per_iter (device, iters int32; either may be NULL). */
typedef struct {
  int32_t autotune;        /* 1: time candidate segment sizes and loads in flight at creation */
  int32_t px_per_thread;   /* segment = 256 * px_per_thread pixels (4, 8, 16, 32 or 64; 0 = 16) when not
                              autotuning */
  int32_t use_graph;       /* 1: capture the iterations in hipGraphs (default), 0: direct launches */
  ds3_timer* reduce_timer; /* may be NULL: recorded around the fused residual/Hessian launch of the last
                              iteration of every ds3_gn_plan_run, which then runs as direct launches
                              instead of a graph replay (same kernels, same results) */
  int32_t unroll;          /* match records in flight per thread (1, 2 or 4; 0 = 2) when not autotuning */
  int32_t solver;          /* normal equations of eq. (7): 1 = the dense solver (ds3_chol_ladder_solve);
                              2 = the block-sparse solver of the plan's keyframe-pair pattern
                              (ds3_spchol_*; DS3_ENOSPACE when the pattern does not fit it); 3 = the
                              tile-sparse solver of that pattern (ds3_tilechol_*); 0 (the default) = the
                              tile-sparse solver when its elimination tree has fewer levels than the
                              dense solver has 32-row panels, else the dense one. All run the same
                              epsilon ladder. */
} ds3_plan_opts;

int ds3_gn_plan_create(int32_t n_kf, const ds3_image* kf, const void* xyzc_arena, ds3_dtype dtype,
                       const ds3_edge* edges, int32_t n_edges, const int32_t* idx_arena,
                       const ds3_gn_params* params, const int32_t* anchors, int32_t n_anchors,
                       const ds3_plan_opts* opts, double* poses, void** plan_out, void* stream);
int ds3_gn_plan_run(void* plan, int32_t iters, double* cost_per_iter, int32_t* status_per_iter,
                    void* stream);
/* Re-gathers the match stream from the current idx arena and keyframe arena (one launch on `stream`, no
 * synchronisation; same topology). Needed after either arena changes. */
int ds3_gn_plan_refresh(void* plan, void* stream);
/* Replaces the plan's reduce_timer (NULL: none) for the following runs; the caller keeps it alive. */
int ds3_gn_plan_set_timer(void* plan, ds3_timer* timer);
/* Timing hook for the fused residual/Hessian kernel alone: launches it `reps` times on `stream` at the
 * plan's current poses (device prep included), bracketed by events; *ms_out (host) = mean ms per
 * launch. Synchronises. */
int ds3_gn_plan_time_reduce(void* plan, int32_t reps, float* ms_out, void* stream);
/* Plan facts at creation (host, the first n_info of): [segments, px_per_thread, px of j scanned over all
 * edges, valid matches (idx in range), bytes of the streaming model (4 B idx per scanned px + both arena
 * entries per valid match), bytes the residual kernel reads per iteration (records + segment counts),
 * bytes one ds3_gn_plan_refresh moves (idx + both entries read, records written), records in flight per
 * thread, solver (1 dense, 2 block-sparse, 3 tile-sparse), blocks (block-sparse) or 32x32 tiles
 * (tile-sparse) of the sparse factor (0 for dense), levels of its elimination tree (0 for dense)]. */
int ds3_gn_plan_info(void* plan, int64_t* info, int32_t n_info);
int ds3_gn_plan_destroy(void* plan);
/* The autotuner's cache: one line per (device, dtype, shape mix) with the tile shape it picked, in the
 * file named by the environment variable DS3_TUNE_CACHE, else $HOME/.cache/ds3_tune.txt. Host only (no
 * GPU call): creates the file's directory if it is missing (mkdir, no child process) and removes the
 * file, so that the next plan with opts->autotune times its candidates again. DS3_EINVAL if the file
 * exists and cannot be removed. */
int ds3_tune_cache_reset(void);

/* ---------------------------------------------------------------------------------------------------
 * Ray-range tracking (Sec. III-A: E_track with LM damping, eq. 7 with lambda > 0)
 * ------------------------------------------------------------------------------------------------- */

/* LM schedule of the tracker (the paper states only that the tracker uses LM damping; these values are
 * readings): lambda0 = 1e-4, lambda <- max(lambda * lambda_down, lambda_min) after an accepted trial
 * (lambda_down = 0.1, lambda_min = 1e-9), lambda <- lambda * lambda_up after a rejected one
 * (lambda_up = 10), at most max_trials = 20 trial steps, stop after an accepted step whose largest
 * tangent component is below step_tol = 1e-7. */
typedef struct {
  double lambda0, lambda_min, lambda_up, lambda_down;
  int32_t max_trials;
  double step_tol;
} ds3_track_params;
void ds3_default_track_params(ds3_track_params* p);

/* One tracking problem: a frame's pointmap (image `frame` of the arena) against a keyframe's canonical
 * pointmap (image `keyframe`); its matches are H_f*W_f int32 entries at idx_offset of an idx arena:
 * entry n is the keyframe pixel m matched to frame pixel n, or -1. */
typedef struct {
  ds3_image keyframe;
  ds3_image frame;
  int64_t idx_offset;
} ds3_track_problem;

/* Workspace bytes of ds3_track for these problems (host table) at this dtype. */
size_t ds3_track_workspace_bytes(int32_t n, const ds3_track_problem* probs, ds3_dtype dtype);

/* For each of n independent problems (host table), the pose T_kf (device, n x 8 float64, in: start,
 * out: result) mapping the frame's camera into the keyframe's that minimises
 *   E_track(T_kf) = sum_{(m,n)} sum_c rho([Sigma_mn^-1/2 e_mn(T_kf)]_c),
 * e of eq. (1) with X^j_j = the frame's point, X-hat^i_i = the keyframe's point, Sigma_mn = Sigma / q_mn,
 * q_mn = sqrt(C_k[m] C_f[n]), component-wise Huber rho and IRLS weights (gn: sigma_ray, sigma_dist,
 * huber_k, and the epsilon ladder eps0, eps_mult, max_attempts of eq. 7; gn->lambda is not used). LM:
 * at the kept pose T with IRLS normal equations H, g, a trial solves (H + lambda diag H + eps_r I) tau =
 * -g and T' = Exp(tau) T; it is accepted iff E_track(T') < E_track(T) (schedule in tp), with E_track
 * evaluated in float64 from the stored values for this test (H and g are accumulated in float32; a float32
 * cost cannot resolve the decrease of the last steps before the optimum). Matches with a hole, a
 * non-finite value or a negative confidence product are skipped.
 * Outputs (device): cost_out (n float64) = E_track at the returned pose, trials_out (n int32) = trial
 * steps taken, status_out (n int32, may be NULL) = ladder attempt of the last solve (-1: zero step).
 * One call gathers the matches once, then runs 1 + max_trials rounds of two launches (reduction at the
 * trial poses, LM step) with no host synchronisation; stopped problems are skipped. reduce_timer (may be
 * NULL) is recorded around the first reduction launch (every problem active). Workspace from
 * ds3_track_workspace_bytes. */
int ds3_track(const void* arena, ds3_dtype dtype, const ds3_track_problem* probs, int32_t n,
              const int32_t* idx_arena, const ds3_gn_params* gn, const ds3_track_params* tp, double* T,
              double* cost_out, int32_t* trials_out, int32_t* status_out, ds3_timer* reduce_timer,
              void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): ds3_track without a workspace argument. Its scratch (edge table, match
 * stream, partials, LM states) is a static device array of DS3_TRACK_SCRATCH_BYTES (64 MiB) compiled
 * into the library: each GPU the library runs on holds its own copy until the process ends, and the call
 * itself allocates nothing (no hipMalloc, no library allocation). Problems whose scratch exceeds that size
 * (ds3_track_workspace_bytes reports it; about 6.4 MB per 512x384 frame in f32, 3.2 MB in bf16) are
 * rejected with DS3_ENOSPACE and nothing is launched. Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (two host threads, or two streams whose work is in flight together)
 * race and give undefined results; calls ordered on one stream are safe. No reduce timer. Arguments,
 * outputs and errors otherwise as ds3_track. */
#define DS3_TRACK_SCRATCH_BYTES (64u << 20)
int ds3_track_noalloc(const void* arena, ds3_dtype dtype, const ds3_track_problem* probs, int32_t n,
                      const int32_t* idx_arena, const ds3_gn_params* gn, const ds3_track_params* tp, double* T,
                      double* cost_out, int32_t* trials_out, int32_t* status_out, void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Terminal segment-level depth refinement (Sec. III-E, eqs. 8-10)
 * ------------------------------------------------------------------------------------------------- */

/* Constants: M_k segments per keyframe (about 200), C_min = 1.5, 16 pixels per segment at least,
 * sigma_point = 0.05, lambda_smooth = lambda_prior = 1, lambda_lm = 0.05, eta_max = 0.5 (Sec. III-E); the
 * SLIC iteration count (10) and the Huber kappa of the point residual (the pose cost's 1.345) are readings. */
typedef struct {
  int32_t segments_per_kf;
  double conf_min;
  int32_t min_seg_px, slic_iters;
  double sigma_point, huber_k, lambda_smooth, lambda_prior, lambda_lm, eta_max;
} ds3_depth_params;
void ds3_default_depth_params(ds3_depth_params* p);

/* Creates a refinement plan over the pristine keyframe arena (the X_init snapshot of eq. 8; caller's, must
 * outlive the plan and stay unchanged), the graph's edges and matches (idx arena as for the graph step;
 * caller's) and the anchor keyframes (host list; their segments stay fixed). Creation segments every
 * keyframe on the device (SLIC over quantised normals and normalised log-range in exact integer arithmetic:
 * F = (round(1024 (n + 1)) x3, round(1024 l)), S = round(sqrt(HW / M_k)), D = S^2 |dF|^2 + 512^2 |dxy|^2
 * over the 3x3 neighbouring cells' centres, ties to the lowest index, centres to the floor of their members'
 * mean), excludes pixels below conf_min and segments below min_seg_px, builds the boundary table (4-adjacent
 * pixel pairs of two valid segments, mean log-range difference) and sets eta = 0. Segment ids are global:
 * keyframe k owns ids [base_k, base_k + nx_k ny_k), nx_k ny_k <= 256 (else DS3_EINVAL). The plan owns its
 * device buffers (labels 4 B and features 8 B per arena pixel, 2 x 49 x 12 B boundary slots and a few
 * doubles per segment); creation synchronises once. */
int ds3_depth_plan_create(int32_t n_kf, const ds3_image* kf, const void* arena, ds3_dtype dtype,
                          const ds3_edge* edges, int32_t n_edges, const int32_t* idx_arena, const int32_t* anchors,
                          int32_t n_anchors, const ds3_depth_params* params, void** plan_out, void* stream);
/* iters Jacobi-style damped Newton steps with the poses fixed (device, n_kf x 8): per segment the diagonal
 * of the data term's normal equations (J_g = -X_i(eta), J_h = sR_ij X_j(eta), whitened by
 * sqrt(q)/sigma_point, Huber weights), lambda_smooth per boundary pair and lambda_prior, the full gradient
 * of E' = sum rho + (lambda_smooth/2) sum_B ((eta_g - eta_h) + Delta_gh)^2 + (lambda_prior/2) sum eta^2,
 * step = clip(-g / ((1 + lambda_lm) H), +-eta_max); anchor segments fixed. cost_per_iter (device, iters
 * float64, may be NULL) = E' at each iteration's input eta. data_timer (may be NULL) brackets the data-term
 * launch of the last iteration. No host synchronisation. iters <= 1024. */
int ds3_depth_plan_run(void* plan, const double* poses, int32_t iters, double* cost_per_iter, ds3_timer* data_timer,
                       void* stream);
/* [segment slots, valid segments, boundary slots in use (each unordered pair twice), data-kernel tiles,
 * pixels of j scanned per iteration over all edges, arena pixels] */
int ds3_depth_plan_info(void* plan, int64_t* info, int32_t n_info);
/* Device copies: labels_out (arena pixels, int32: global segment id or -1), eta_out (segment slots, float64);
 * either may be NULL. */
int ds3_depth_plan_get(void* plan, int32_t* labels_out, double* eta_out, void* stream);
/* Replaces eta (device, segment slots, float64). */
int ds3_depth_plan_set_eta(void* plan, const double* eta, void* stream);
/* The refined pointmaps of eq. (8), X_init exp(eta_g) per pixel (excluded pixels unchanged), as a float32
 * xyzc arena (device, 16 B aligned, arena pixels x 4; the confidences copied). */
int ds3_depth_plan_apply(void* plan, float* xyzc_out, void* stream);
int ds3_depth_plan_destroy(void* plan);

/* ---------------------------------------------------------------------------------------------------
 * Cost and its adjoint (gradient of eq. 5 with the matches held fixed)
 * ------------------------------------------------------------------------------------------------- */

/* E_global at poses (device float64 scalar): one launch over every (edge, tile) pair evaluates the Huber
 * cost of each valid match (float32 per block, float64 per edge, fixed summation order, so the result
 * is reproducible), no Jacobians. */
int ds3_gn_cost(const double* poses, int32_t n_kf, const ds3_image* kf, const void* xyzc_arena,
                ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges, const int32_t* idx_arena,
                const ds3_gn_params* params, double* cost_out, void* workspace, size_t ws_bytes,
                void* stream);

/* dE/dX and dE/dC per arena pixel (device float32, 3 resp. 1 per pixel) and dE/dtau per keyframe (device
 * float64 n_kf x 7), all scaled by dcost (host float) and all OVERWRITTEN for every pixel of every
 * keyframe in kf (arena pixels outside the keyframes are left untouched). Two per-pixel launches: the
 * query side is gathered per keyframe and stored, then the gathered side adds its terms with float
 * atomics, so the per-pixel sums are not bitwise reproducible. adjoint_timer (may be NULL) is recorded
 * around the two per-pixel launches. */
int ds3_gn_cost_adjoint(const double* poses, int32_t n_kf, const ds3_image* kf, const void* xyzc_arena,
                        ds3_dtype dtype, const ds3_edge* edges, int32_t n_edges,
                        const int32_t* idx_arena, const ds3_gn_params* params, float dcost,
                        float* grad_xyz, float* grad_conf, double* grad_tau, ds3_timer* adjoint_timer,
                        void* workspace, size_t ws_bytes, void* stream);

/* Cost + adjoint plan for a graph whose matches stay fixed (the contents of xyzc_arena and the poses may
 * change between runs; idx_arena and the topology must not). Creation inverts every match map on the
 * device: for edge e and pixel m of keyframe i(e), the pixels n of j(e) with idx[n] = m in increasing n
 * (CSR). It allocates device memory (about 4 B per pixel of i(e) plus 4 B per pixel of j(e), per edge)
 * and a temporary count array of 4 B per pixel of i(e) per edge, freed before it returns; it
 * synchronises the stream. *plan_out (host) receives the plan, NULL on failure. */
int ds3_adjoint_plan_create(int32_t n_kf, const ds3_image* kf, const void* xyzc_arena, ds3_dtype dtype,
                            const ds3_edge* edges, int32_t n_edges, const int32_t* idx_arena,
                            const ds3_gn_params* params, void** plan_out, void* stream);
/* One pass over the graph at poses (device n_kf x 8): E_global into *cost_out (device float64 scalar, may
 * be NULL) and the gradients of ds3_gn_cost_adjoint (same layouts, scaled by dcost, overwritten), with
 * both sides of every pixel gathered in a fixed order and stored once: no atomics, bitwise reproducible.
 * timer (may be NULL) is recorded around the per-pixel launch. Runs on one plan must not overlap. */
int ds3_adjoint_plan_run(void* plan, const double* poses, float dcost, float* grad_xyz, float* grad_conf,
                         double* grad_tau, double* cost_out, ds3_timer* timer, void* stream);
int ds3_adjoint_plan_destroy(void* plan);

/* ---------------------------------------------------------------------------------------------------
 * Canonical pointmap fusion (Sec. III-A, eq. 2)
 * ------------------------------------------------------------------------------------------------- */

/* One registered prediction to fuse into a keyframe's canonical pointmap: n_px pixels starting at pixel
 * canon_off of the canonical arena and at pixel pred_off of the prediction arena. */
typedef struct {
  int64_t canon_off;
  int64_t pred_off;
  int64_t n_px;
} ds3_fuse_pair;

/* Workspace bytes of ds3_fuse for n_pairs pairs (the pair table on the device). */
size_t ds3_fuse_workspace_bytes(int32_t n_pairs);

/* The confidence-weighted running average of eq. (2) for n_pairs (keyframe, frame) pairs in one launch.
 * For pair p and pixel m < pairs[p].n_px, with c = canon[canon_off + m] (xyz: canonical point X-hat of
 * the keyframe, w: its confidence C-hat) and x = pred[pred_off + m] (xyz: the frame's prediction of the
 * same keyframe pixel in the frame's camera, w: its confidence C):
 *   y = T_p x,   X-hat <- (C-hat X-hat + C y) / (C-hat + C),   C-hat <- C-hat + C,
 * evaluated in float64 from the float32 inputs and rounded once to float32.
 *   canon (device, n_canon_px float4 xyzc pixels, updated in place); pred (device, n_pred_px float4
 *   xyzc pixels; it may not overlap canon); T (device, n_T >= n_pairs poses of 8 float64 in the pose
 *   layout, T_p = T_kf mapping the frame into the keyframe); pairs (host, n_pairs entries). Every pair
 *   must lie inside both arenas (DS3_EINVAL otherwise, checked on the host before any launch).
 * A pixel whose prediction has a non-finite entry, or whose summed confidence is not positive, is left
 * unchanged. Two pairs may not share a canonical pixel (checked on the host: DS3_EINVAL), since they
 * would race within the launch; fuse them in separate calls in their order. n_pairs = 0 is a no-op.
 * Workspace from ds3_fuse_workspace_bytes. */
int ds3_fuse(float* canon, int64_t n_canon_px, const float* pred, int64_t n_pred_px,
             const ds3_fuse_pair* pairs, int32_t n_pairs, const double* T, int32_t n_T, void* workspace,
             size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DS3_H */
