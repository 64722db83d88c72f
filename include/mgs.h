/*
 * mgs.h -- C ABI of the MI355X (gfx950) order-independent Gaussian splatting pass.
 *
 * The pass renders 3D Gaussians (mean, scale, rotation, opacity, first-order SH
 * colour; Appendix B of Mobile-GS, arXiv 2603.11531) with the paper's sort-free,
 * depth-aware order-independent blend (Sec. 3.1, Eq. 2 and Eq. 3) and its
 * view-dependent enhancement MLP (Eq. 4).  A conventional sorted alpha-blend
 * path (Eq. 11) is provided for comparison.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array pointers are DEVICE pointers unless stated otherwise; struct
 *   arguments themselves (mgs_camera, mgs_gaussians, ...) are HOST structs read
 *   during the call only.
 * - The caller owns all device memory.  The library never allocates or frees
 *   device memory and keeps no mutable global state; calls on different streams
 *   are independent.
 * - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default
 *   stream).  MGS_OK means "validated and enqueued"; buffers must stay valid
 *   until the stream reaches the work.
 * - Per-Gaussian inputs are structure-of-arrays float32 ("[3][n]" = three
 *   planes of n floats).  Images are planar float32 [3][H][W].
 * - Pixel (i, j) has its centre at (i + 0.5, j + 0.5); camera space is
 *   x right, y down, z forward; x_c = R * x_world + t.
 * - Tiles are 16 x 16 pixels, numbered row-major t = ty * tiles_x + tx with
 *   tiles_x = ceil(W / 16), tiles_y = ceil(H / 16).
 * - Return codes: MGS_OK (0) or a negative MGS_ERR_*; no exception crosses the
 *   ABI.  mgs_last_error() returns a thread-local description of the last error.
 */
#ifndef MGS_H
#define MGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGS_OK                 0
#define MGS_ERR_INVALID_ARG   (-1)  /* NULL required pointer, bad size, misaligned pointer */
#define MGS_ERR_CAPACITY      (-2)  /* pair count exceeded the caller's capacity           */
#define MGS_ERR_HIP           (-3)  /* a HIP launch or runtime call failed                 */
#define MGS_ERR_UNSUPPORTED   (-4)  /* valid but not supported (e.g. tile size != 16)      */

#define MGS_TILE        16
#define MGS_MLP_IN      22          /* [P_i(3), s_i(3), r_i(4), Y_i(12)]                  */
#define MGS_MLP_HIDDEN  64
/* Bytes of the packed enhancement-MLP weights written by mgs_mlp_pack. */
#define MGS_MLP_PACKED_BYTES 15360
/* Floats per projected Gaussian record ("splat"), see mgs_projected. */
#define MGS_SPLAT_FLOATS 12

/* Per-Gaussian blending weight w (mgs_project_weighted / mgs_enhance_project_weighted):
 * Eq. 3, or the two ablations of it in the paper's ablation table (Table 3), read as
 * d = 1 ("without depth") and the exp(s_max / d) term dropped ("without scale"). */
#define MGS_WEIGHT_EQ3       0      /* w = phi^2 + phi/d^2 + exp(s_max/d)                */
#define MGS_WEIGHT_NO_DEPTH  1      /* w = phi^2 + phi + exp(s_max)                      */
#define MGS_WEIGHT_NO_SCALE  2      /* w = phi^2 + phi/d^2                               */
/* The weighting function of the SortFreeGS composite the paper builds on (Eq. 1, Sec. 2):
 * w = exp(-sigma_i d^beta_i) with per-Gaussian sigma_i, beta_i; selected only through
 * mgs_project_sortfree / mgs_enhance_project_sortfree, which take the two arrays. */
#define MGS_WEIGHT_SORTFREE  3      /* w = exp(-sigma_i d^beta_i)                        */

/* Pinhole camera.  R is row-major world->camera (rows: right, down, forward). */
typedef struct mgs_camera {
    float   R[9];
    float   t[3];
    float   fx, fy, cx, cy;
    int32_t width, height;
    float   near_z;           /* Gaussians with camera depth <= near_z are culled */
} mgs_camera;

/* Gaussian attributes (Appendix B), SoA float32 device arrays. */
typedef struct mgs_gaussians {
    int64_t      n;
    const float *mean;          /* [3][n] world position mu                          */
    const float *log_scale;     /* [3][n] s = exp(log_scale)                          */
    const float *quat;          /* [4][n] rotation (w, x, y, z), need not be unit     */
    const float *opacity_logit; /* [n]    o = sigmoid(opacity_logit)                  */
    const float *sh;            /* [12][n] SH degree-1 coefficients, plane 3k + ch    */
} mgs_gaussians;

/* Gradients with respect to the raw attributes; same layout as mgs_gaussians. */
typedef struct mgs_gaussians_grad {
    float *mean, *log_scale, *quat, *opacity_logit, *sh;
} mgs_gaussians_grad;

/*
 * Projected Gaussians, written by mgs_project.
 *   splat   [n][12] float32, three float4 per Gaussian:
 *             (mx, my, log2(o_eff), w)   screen-space mean, log2 effective opacity, Eq. 3 weight
 *             (kA, beta, kG, depth)      the exponent of Eq. 2 as two non-negative parts:
 *                                        log2(alpha) = log2(o_eff) + kA t^2 + kG dy^2,
 *                                        t = dx + beta dy, (dx, dy) = pixel - mean, and for the
 *                                        2D covariance [[a, b], [b, c]] (determinant det):
 *                                        kA = -(1/2) log2(e) c / det, beta = -b / c,
 *                                        kG = -(1/2) log2(e) / c; depth = camera z
 *             (r, g, b, o_eff)           SH colour, effective opacity
 *   rect    [n][2] uint32: (tx0 | ty0 << 16, tx1 | ty1 << 16), inclusive tile range
 *   n_tiles [n] uint32: tiles covered (0 = culled)
 * Pointers must be 16-byte aligned (splat) / 8-byte (rect) / 4-byte (n_tiles).
 */
typedef struct mgs_projected {
    float    *splat;
    uint32_t *rect;
    uint32_t *n_tiles;
} mgs_projected;

/* Thread-local message of the last error (static storage, never NULL). */
const char *mgs_last_error(void);

/*
 * Checked builds.  libmgs_checked.so is this library built with MGS_CHECK_BOUNDS: its kernels
 * check the indices they derive (list positions and writes against the pair count and capacity,
 * rectangles against the tile grid, split-blend items and backward slots against their
 * workspace bounds, pruning's survivor and gather indices); a failed check skips the access and
 * sets a bit (MGS_BOUNDS_*).
 * mgs_bounds_checked: 1 in a checked build, else 0.
 * mgs_bounds_status: synchronises the device, writes the OR of the bits set since the last
 * clear to *flags (always 0 in an unchecked build) and, if `clear`, clears them.
 */
#define MGS_BOUNDS_EXPAND_WRITE 0x01u
#define MGS_BOUNDS_RECT_GRID    0x02u
#define MGS_BOUNDS_LIST_WRITE   0x04u
#define MGS_BOUNDS_LIST_READ    0x08u
#define MGS_BOUNDS_SPLIT_ITEM   0x10u
#define MGS_BOUNDS_BWD_SLOT     0x20u
#define MGS_BOUNDS_BWD_ITEM     0x40u
#define MGS_BOUNDS_PRUNE_INDEX  0x80u
int mgs_bounds_checked(void);
int mgs_bounds_status(uint32_t *flags, int clear);
/* Library version string. */
const char *mgs_version(void);

/*
 * Enhancement-MLP parameters (Eq. 4), one contiguous float32 array of
 * MGS_MLP_PARAMS values, row-major [out][in] matrices:
 *   W1 [64][22] @ MGS_MLP_OFF_W1, b1 [64] @ MGS_MLP_OFF_B1, W2 [64][64] @ MGS_MLP_OFF_W2,
 *   b2 [64] @ MGS_MLP_OFF_B2, w_phi [64] @ MGS_MLP_OFF_WPHI, b_phi @ MGS_MLP_OFF_BPHI,
 *   w_o [64] @ MGS_MLP_OFF_WO, b_o @ MGS_MLP_OFF_BO.
 * The network is F = ReLU(W2 ReLU(W1 x + b1) + b2), phi = ReLU(w_phi . F + b_phi),
 * m = sigmoid(w_o . F + b_o), x = [P_i, s_i, r_i, Y_i].  Gradients use the same layout.
 */
#define MGS_MLP_OFF_W1    0
#define MGS_MLP_OFF_B1    1408
#define MGS_MLP_OFF_W2    1472
#define MGS_MLP_OFF_B2    5568
#define MGS_MLP_OFF_WPHI  5632
#define MGS_MLP_OFF_BPHI  5696
#define MGS_MLP_OFF_WO    5697
#define MGS_MLP_OFF_BO    5761
#define MGS_MLP_PARAMS    5762

/*
 * mgs_mlp_pack -- MLP parameters -> packed bfloat16 MFMA operands for mgs_enhance.
 * In: params (device, MGS_MLP_PARAMS floats).  Out: `packed`, MGS_MLP_PACKED_BYTES
 * bytes of device memory, 16-byte aligned.  Weights are rounded to bfloat16
 * (nearest-even); biases stay float32.  Re-run after every weight update.
 */
int mgs_mlp_pack(const float *params, void *packed, void *stream);

/*
 * The appendix's enhancement network MLP_f: ReLU hidden layers of 256, 128 and 64 neurons
 * (Additional Implementation Details), with the inputs x and the phi / opacity heads of
 * Eq. 4 above.  Parameters: one float32 array of MGS_MLPF_PARAMS values, row-major:
 *   W1 [256][22], b1 [256], W2 [128][256], b2 [128], W3 [64][128], b3 [64],
 *   w_phi [64], b_phi, w_o [64], b_o  (offsets MGS_MLPF_OFF_*).
 */
#define MGS_MLPF_OFF_W1    0
#define MGS_MLPF_OFF_B1    5632
#define MGS_MLPF_OFF_W2    5888
#define MGS_MLPF_OFF_B2    38656
#define MGS_MLPF_OFF_W3    38784
#define MGS_MLPF_OFF_B3    46976
#define MGS_MLPF_OFF_WPHI  47040
#define MGS_MLPF_OFF_BPHI  47104
#define MGS_MLPF_OFF_WO    47105
#define MGS_MLPF_OFF_BO    47169
#define MGS_MLPF_PARAMS    47170
/* Bytes of the packed MLP_f written by mgs_mlp_f_pack (bf16 MFMA operands + float32 biases). */
#define MGS_MLPF_PACKED_BYTES 104208

/*
 * mgs_mlp_f_pack -- MLP_f parameters (device, MGS_MLPF_PARAMS floats) -> packed operands
 * for mgs_enhance_project_mlp_f (`packed`: MGS_MLPF_PACKED_BYTES bytes of device memory,
 * 16-byte aligned).  Weights are rounded to bfloat16 (nearest-even), biases stay float32.
 */
int mgs_mlp_f_pack(const float *params, void *packed, void *stream);

/*
 * mgs_enhance_project_mlp_f -- mgs_enhance_project with MLP_f in place of the two-layer
 * network: per Gaussian phi and omod from MLP_f (bfloat16 products, float32
 * accumulation), then the projection of mgs_project.  Same outputs and argument rules as
 * mgs_enhance_project; `packed_mlp_f` from mgs_mlp_f_pack.  The backward pass
 * (mgs_render_backward) differentiates the two-layer network only.
 */
int mgs_enhance_project_mlp_f(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp_f, int tile,
                              float alpha_min, mgs_projected *out, float *phi, float *omod, void *stream);

/*
 * mgs_enhance -- view-dependent enhancement, Eq. 4 (Sec. 3.1).
 * For every Gaussian: P_i = (mu - t_v)/|mu - t_v| with t_v the camera centre,
 * s = exp(log_scale), r = normalised quaternion, Y = SH coefficients; runs the
 * packed MLP with bfloat16 inputs and float32 accumulation.
 * Out: phi [n] (>= 0) and omod [n] (in (0, 1)), float32 device arrays.
 * The opacity head modulates the stored opacity: o_eff = sigmoid(logit) * omod.
 */
int mgs_enhance(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp,
                float *phi, float *omod, void *stream);

/*
 * mgs_project -- per-Gaussian preprocessing for Eq. 2 / Eq. 3.
 * Camera-space depth d, EWA projection Sigma' = J W Sigma W^T J^T + 0.3 I of
 * Sigma = R S S^T R^T (J clamped to 1.3x the half field of view), first-order
 * SH colour c = max(0, 1/2 + C0 Y0 + C1 (-P_y Y1 + P_z Y2 - P_x Y3)),
 * o_eff = sigmoid(logit) * omod, weight w = phi^2 + phi/d^2 + exp(s_max/d)
 * (Eq. 3), and the inclusive tile rectangle of the pixel centres inside the
 * bounding box of {alpha >= alpha_min}.
 * phi / omod may be NULL (then phi = 1, omod = 1: the MLP's initial state).
 * Culled (n_tiles = 0): d <= near_z, o_eff < alpha_min, empty pixel range.
 * tile must be MGS_TILE.  alpha_min in (0, 1).
 */
int mgs_project(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                const float *omod, int tile, float alpha_min, mgs_projected *out,
                void *stream);

/*
 * mgs_project_weighted -- mgs_project with the weight w of weight_mode (MGS_WEIGHT_*,
 * the Eq. 3 ablations of Table 3); mgs_project is weight_mode = MGS_WEIGHT_EQ3.  Every
 * other output is the same.  An unknown weight_mode is MGS_ERR_INVALID_ARG.  The
 * backward pass (mgs_render_backward) differentiates Eq. 3 only.
 */
int mgs_project_weighted(const mgs_gaussians *g, const mgs_camera *cam, const float *phi,
                         const float *omod, int tile, float alpha_min, int weight_mode,
                         mgs_projected *out, void *stream);

/*
 * mgs_enhance_project -- mgs_enhance followed by mgs_project in one pass over the
 * attributes (each Gaussian is read once; the MLP runs on MFMA per 64-Gaussian
 * wave).  Writes the same projected record as the two calls, and phi / omod
 * (needed by mgs_render_backward).
 */
int mgs_enhance_project(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp, int tile,
                        float alpha_min, mgs_projected *out, float *phi, float *omod, void *stream);

/*
 * mgs_enhance_project_sh -- mgs_enhance_project for a scene whose colour is real SH of order
 * sh_degree (0..3; Table 3's SH-order variants): g->sh holds 3 (sh_degree + 1)^2 planes,
 * plane 3 k + channel, k = l^2 + l + m (orders m = -l..l, sign (-1)^m on odd m, as the
 * first-order terms above).  Colour c = max(0, 1/2 + sum_k Y_k(P) sh_k); the MLP input Y_i is
 * the order <= 1 block (zeros for order 0).  sh_degree 1 is mgs_enhance_project.  Other
 * arguments and outputs as mgs_enhance_project; sh_degree outside 0..3 is MGS_ERR_INVALID_ARG.
 * The backward pass (mgs_render_backward) is first-order only.
 */
int mgs_enhance_project_sh(const mgs_gaussians *g, int sh_degree, const mgs_camera *cam, const void *packed_mlp,
                           int tile, float alpha_min, mgs_projected *out, float *phi, float *omod, void *stream);

/*
 * mgs_enhance_project_weighted -- mgs_enhance_project with the weight of weight_mode
 * (MGS_WEIGHT_*, as mgs_project_weighted).
 */
int mgs_enhance_project_weighted(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp,
                                 int tile, float alpha_min, int weight_mode, mgs_projected *out, float *phi,
                                 float *omod, void *stream);

/*
 * SortFreeGS weighting (Eq. 1, Sec. 2), the sort-free composite the paper compares its own
 * against:  C = (c_bg w_bg + sum_i c_i alpha_i w(d_i)) / (w_bg + sum_i alpha_i w(d_i)),
 * w(d_i) = exp(-sigma_i d_i^beta_i), d_i the camera depth.  It has no transmittance term.
 *
 * mgs_project_sortfree -- mgs_project with w = exp(-sigma_i d_i^beta_i) in the splat record's
 * weight slot (MGS_WEIGHT_SORTFREE); sigma, beta: device float32 [n] (required for n > 0).
 * phi plays no part in this weight; omod (NULL -> 1) still modulates the opacity.
 * mgs_enhance_project_sortfree -- the same after the enhancement MLP (phi / omod written as
 * by mgs_enhance_project; only omod enters the record).  Other arguments and errors as
 * mgs_project / mgs_enhance_project.  mgs_render_backward does not differentiate Eq. 1.
 */
int mgs_project_sortfree(const mgs_gaussians *g, const mgs_camera *cam, const float *omod, const float *sigma,
                         const float *beta, int tile, float alpha_min, mgs_projected *out, void *stream);
int mgs_enhance_project_sortfree(const mgs_gaussians *g, const mgs_camera *cam, const void *packed_mlp,
                                 const float *sigma, const float *beta, int tile, float alpha_min,
                                 mgs_projected *out, float *phi, float *omod, void *stream);

/*
 * Vector-quantised Gaussians (Sec. 3.2, neural vector quantization: attribute
 * sub-vectors, each with its own codebook; five groups and 2^10 codewords per
 * codebook in the paper's deployed configuration).  Positions stay float32.  The 20
 * other attributes, in the order [log_scale(3), quat(4) w,x,y,z, opacity_logit,
 * sh(12) plane 3k+ch], are five consecutive sub-vectors of four values: attribute
 * value j of group g of Gaussian i is codebooks[(g * MGS_NVQ_CODEWORDS + codes[g * n + i]) * 4 + j].
 * Codes are taken modulo MGS_NVQ_CODEWORDS, so no code can read outside the codebooks.
 * Device pointers: mean [3][n] float32, codes [5][n] uint16, codebooks
 * [5][1024][4] float32 (16-byte aligned; the caller owns all of them).
 */
#define MGS_NVQ_GROUPS    5
#define MGS_NVQ_DIM       4
#define MGS_NVQ_CODEWORDS 1024

typedef struct mgs_gaussians_nvq {
    int64_t n;
    const float *mean;
    const uint16_t *codes;
    const float *codebooks;
} mgs_gaussians_nvq;

/*
 * mgs_nvq_decode -- the codebook lookup above, written out as the float32 SoA planes
 * of mgs_gaussians (log_scale [3][n], quat [4][n], opacity_logit [n], sh [12][n];
 * device, caller-owned).  Bit-exact copies of the codewords.
 */
int mgs_nvq_decode(const mgs_gaussians_nvq *q, float *log_scale, float *quat, float *opacity_logit, float *sh,
                   void *stream);

/*
 * mgs_enhance_project_nvq -- mgs_enhance_project reading the attributes through the
 * codebooks (22 bytes per Gaussian from memory: mean and codes; the 80 KB of
 * codebooks stay in cache).  Same outputs, bit for bit, as mgs_enhance_project on
 * the decoded attributes.  packed_mlp as for mgs_enhance (required).
 */
int mgs_enhance_project_nvq(const mgs_gaussians_nvq *q, const mgs_camera *cam, const void *packed_mlp, int tile,
                            float alpha_min, mgs_projected *out, float *phi, float *omod, void *stream);

/*
 * mgs_bin_workspace -- device workspace bytes mgs_bin needs for n Gaussians,
 * a tile grid of tiles_x * tiles_y and at most `capacity` tile/Gaussian pairs.
 */
int mgs_bin_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes);

/*
 * mgs_bin -- tile binning with no depth sort (atomic-free prefix sums).
 * From rect / n_tiles of mgs_project: P = sum(n_tiles) pairs are laid out per
 * tile; the list of tile t is gids[tile_offsets[t] .. tile_offsets[t+1]) in
 * ascending Gaussian index.  The result is deterministic (bit-identical runs).
 * Out: tile_offsets [T + 1] uint32, gids [capacity] uint32, n_pairs [1]
 * uint32 (device) = P.  If P > capacity nothing but n_pairs is written; the
 * caller detects the overflow from n_pairs after synchronising (this keeps
 * the call free of host synchronisation).
 * ws/ws_bytes: workspace of at least mgs_bin_workspace() bytes, 256-byte aligned.
 * MGS_ERR_INVALID_ARG for a grid of 2^20 or more 8x8-tile supertiles.
 */
int mgs_bin(const mgs_projected *proj, int64_t n, int tiles_x, int tiles_y, void *ws,
            size_t ws_bytes, uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity,
            uint32_t *n_pairs, void *stream);

/*
 * mgs_check_capacity -- the caller's overflow check after mgs_bin / mgs_bin_sorted (the tile
 * lists that the per-pixel sums of Eq. 2, Sec. 3.1, run over).  Waits for `stream`, reads the
 * pair count P that the binning wrote to n_pairs (device, 1 uint32), stores it in *pairs (host;
 * may be NULL) and returns MGS_ERR_CAPACITY when P > capacity (then the lists were not written:
 * re-bin with a workspace and gids for at least P pairs), else MGS_OK.  MGS_ERR_INVALID_ARG for
 * a NULL n_pairs, MGS_ERR_HIP if the stream reports an error.  Synchronises: not for capture.
 */
int mgs_check_capacity(const uint32_t *n_pairs, uint64_t capacity, uint64_t *pairs, void *stream);

/*
 * mgs_blend_oit -- the depth-aware order-independent composite, Eq. 2.
 * For every pixel p over its tile's list: a = o_eff exp(-q/2),
 * q = dx^T Sigma'^-1 dx; pairs with a < alpha_min are skipped;
 * alpha = min(a, alpha_max); N += alpha w c, D += alpha w, T *= (1 - alpha);
 * C = (1 - T) N / D + T bg, or C = bg when no Gaussian contributes.
 * Out: image [3][H][W] float32; aux [5][H][W] float32 = (N/D rgb, D, T) or NULL.
 * bg is a HOST array of 3 floats.
 */
int mgs_blend_oit(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                  const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                  float alpha_max, float *image, float *aux, void *stream);

/*
 * mgs_blend_oit_split -- mgs_blend_oit with long tile lists cut into equal ranges of at
 * most 2048 Gaussians (of about L / 255 for lists longer than 255 x 2048, so a tile has at
 * most 255 ranges), rendered by separate workgroups (the longest first for views of up to
 * 65,536 tiles, in tile order beyond) and merged exactly in range order (Eq. 2's sums are
 * order-independent: N and D add, T multiplies), which balances the work of dense tiles.
 * Results equal mgs_blend_oit up to float32 summation order.
 * n_pairs / capacity: as written / used by mgs_bin (nothing is drawn if n_pairs >
 * capacity).  ws: mgs_blend_oit_split_workspace() bytes, 256-byte aligned.
 * MGS_ERR_INVALID_ARG for a view of 2^24 or more 16x16 tiles.
 */
int mgs_blend_oit_split_workspace(int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes);
int mgs_blend_oit_split(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                        const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, int tile,
                        const float bg[3], float alpha_min, float alpha_max, void *ws, size_t ws_bytes,
                        float *image, float *aux, void *stream);

/*
 * mgs_blend_census -- measurement of the order-independent blend's work on the lists of mgs_bin
 * (not part of rendering).  Writes counts[0] = list entries (tile, Gaussian) P, counts[1] =
 * pixel-Gaussian evaluations the blend executes (64 per 8x8 quadrant its exact quadrant test
 * keeps), counts[2] = pixel-Gaussian pairs that contribute to Eq. 2 (alpha >= alpha_min at the
 * pixel centre, pixels inside the image).  counts: device uint64[3], 8-byte aligned,
 * overwritten.  n_pairs / capacity as for mgs_blend_oit_split (all zero when n_pairs >
 * capacity).  Integer results, independent of scheduling.
 */
int mgs_blend_census(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                     const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, float alpha_min,
                     uint64_t *counts, void *stream);

/*
 * mgs_blend_oit_split_noalloc -- mgs_blend_oit_split without a caller workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a library-owned static device array of
 * MGS_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first use on that GPU until the
 * process ends; the call itself allocates and frees nothing.  Every argument, rule and result
 * is that of mgs_blend_oit_split (same kernels); the current device must be the device of
 * `stream` and of the buffers.  The array's device address is looked up on the first call on
 * each device (a host call, not an allocation).
 * MGS_ERR_CAPACITY (nothing enqueued) when the split blend of this view and capacity needs more
 * workspace than MGS_NOALLOC_SCRATCH_BYTES (mgs_blend_oit_split_workspace reports it; about
 * 10 bytes per unit of capacity: 1600x1063 fits up to ~12.8 M pairs).
 * Calls share their GPU's one array, which keeps the last call's contents: calls that overlap
 * on one GPU (other streams, other host threads) race and must be serialised by the caller.
 */
#define MGS_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
int mgs_blend_oit_split_noalloc(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                                const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, int tile,
                                const float bg[3], float alpha_min, float alpha_max, float *image, float *aux,
                                void *stream);

/*
 * mgs_blend_sortfree / mgs_blend_sortfree_split -- mgs_blend_oit / mgs_blend_oit_split with
 * the composite of Eq. 1 (Sec. 2) in place of Eq. 2's:  C = (bg w_bg + N) / (w_bg + D), with
 * N = sum alpha w c and D = sum alpha w over the same contributors (a >= alpha_min, alpha
 * clamped at alpha_max); C = bg where w_bg + D = 0.  w_bg >= 0 (a host float), otherwise
 * MGS_ERR_INVALID_ARG.  The weights are those of the projected records (normally from
 * mgs_project_sortfree).  aux, when non-NULL, receives (N/D rgb, D, T) as for Eq. 2.  Every
 * other argument, workspace and rule is that of the Eq. 2 call.
 */
int mgs_blend_sortfree(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                       const mgs_camera *cam, int tile, const float bg[3], float w_bg, float alpha_min,
                       float alpha_max, float *image, float *aux, void *stream);
int mgs_blend_sortfree_split(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                             const uint32_t *n_pairs, uint64_t capacity, const mgs_camera *cam, int tile,
                             const float bg[3], float w_bg, float alpha_min, float alpha_max, void *ws,
                             size_t ws_bytes, float *image, float *aux, void *stream);

/*
 * Sorted comparison path (3DGS alpha blending, Eq. 11, Appendix B).
 * mgs_bin_sorted: like mgs_bin but each tile's list is in ascending camera
 * depth (ties by Gaussian index): LSD radix sort of 64-bit (tile << 32 |
 * depth bits) keys.  Same outputs and overflow rule as mgs_bin.
 * mgs_blend_sorted: front-to-back C = sum_k c_k alpha_k T_k + T bg, compositing
 * a contributor only while the transmittance before it is >= t_stop.
 */
int mgs_bin_sorted_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes);
int mgs_bin_sorted(const mgs_projected *proj, int64_t n, int tiles_x, int tiles_y, void *ws,
                   size_t ws_bytes, uint32_t *tile_offsets, uint32_t *gids, uint64_t capacity,
                   uint32_t *n_pairs, void *stream);
int mgs_blend_sorted(const mgs_projected *proj, const uint32_t *tile_offsets, const uint32_t *gids,
                     const mgs_camera *cam, int tile, const float bg[3], float alpha_min,
                     float alpha_max, float t_stop, float *image, void *stream);

/*
 * mgs_tile_sort -- the lists of the sorted comparison path (Eq. 11's front-to-back order) as a
 * segmented sort: each tile list of mgs_bin (ascending Gaussian index) sorted in place by the
 * float32 camera depth of its record, ties by Gaussian index.  The result equals mgs_bin_sorted's
 * lists entry for entry; mgs_blend_sorted then composites them.
 * In: proj / n (the projection mgs_bin read), tile_offsets (device, T + 1 entries), n_pairs
 * (device, mgs_bin's count), capacity (the gids capacity passed to mgs_bin).  In/out: gids
 * (device).  When *n_pairs > capacity (mgs_bin overflowed) nothing is read or written.
 * ws: mgs_tile_sort_workspace() bytes, 256-byte aligned (16 bytes per unit of capacity: the
 * copies through which lists longer than 4,096 entries are sorted).
 */
int mgs_tile_sort_workspace(int tiles_x, int tiles_y, uint64_t capacity, size_t *bytes);
int mgs_tile_sort(const mgs_projected *proj, int64_t n, const uint32_t *tile_offsets, uint32_t *gids,
                  int tiles_x, int tiles_y, uint64_t capacity, const uint32_t *n_pairs, void *ws,
                  size_t ws_bytes, void *stream);

/*
 * mgs_render_backward -- gradients of the OIT pass (Eq. 2, Eq. 3, Eq. 4) with
 * respect to the raw Gaussian attributes and, with the MLP, its parameters.
 * It recomputes per-pixel-pair terms from the forward's aux (N/D rgb, D, T):
 * no per-fragment state is kept.  The reduction over pixels and tiles uses
 * no float atomics, so results are bit-reproducible.
 * In: g, cam, proj / tile_offsets / gids (exactly as used by the forward,
 * capacity = the gids capacity passed to mgs_bin), aux [5][H][W] from
 * mgs_blend_oit, dL_dimage [3][H][W], bg (HOST, 3 floats), alpha_min / alpha_max
 * of the forward.  MLP: mlp_params (MGS_MLP_PARAMS floats, device) plus the
 * forward's phi / omod, or all three NULL when the forward ran without the MLP.
 * Out: *out (same SoA layout as mgs_gaussians, fully overwritten) and, with the
 * MLP, dmlp [MGS_MLP_PARAMS] (overwritten).  The MLP gradient passes straight
 * through the forward's bfloat16 roundings.
 * If the forward's pair count (the sum of proj->n_tiles) exceeds `capacity`, its
 * lists overflowed and were not built: no list is read and every output is zero.
 * ws: mgs_render_backward_workspace() bytes, 256-byte aligned.
 */
int mgs_render_backward_workspace(int64_t n, int tiles_x, int tiles_y, uint64_t capacity, int with_mlp,
                                  size_t *bytes);
int mgs_render_backward(const mgs_gaussians *g, const mgs_camera *cam, const float *mlp_params,
                        const float *phi, const float *omod, const mgs_projected *proj,
                        const uint32_t *tile_offsets, const uint32_t *gids, uint64_t capacity,
                        const float *aux, const float *dL_dimage, const float bg[3], float alpha_min,
                        float alpha_max, void *ws, size_t ws_bytes, mgs_gaussians_grad *out,
                        float *dmlp, void *stream);

/*
 * Batched rendering for serving (several resident scenes, mixed resolutions and
 * poses in one fixed launch sequence).  A request names a resident scene, its
 * packed MLP (or NULL for the MLP's initial state phi = 1, m = 1), a camera,
 * a background and an output image [3][H][W] (device).
 */
typedef struct mgs_request {
    mgs_gaussians g;
    const void   *packed_mlp;
    mgs_camera    cam;
    float         bg[3];
    float        *image;
} mgs_request;

#define MGS_BATCH_MAX_REQUESTS 64

/*
 * mgs_batch_workspace -- bytes of workspace for batches of at most max_gaussians
 * Gaussians in total (each request's count rounded up to a multiple of 256),
 * max_tiles 16x16 tiles in total (1 .. 2^20 - 1), and `capacity` tile/Gaussian pairs
 * in total.
 */
int mgs_batch_workspace(int64_t max_gaussians, int64_t max_tiles, uint64_t capacity, size_t *bytes);

/*
 * mgs_render_batch -- renders every request of a batch with the OIT pass (Eq. 2-4):
 * enhance -> project -> bin -> blend, each one launch for the whole batch.
 * `requests` (device array of mgs_request) and `*n_requests` (device int32,
 * 0..MGS_BATCH_MAX_REQUESTS) are read on the device, and every grid is sized by the
 * limits, so the call enqueues the same work for any batch and can be captured in a
 * hipGraph and replayed after the caller rewrites the request table.
 * Out: each request's image; n_pairs (device uint32) = total pairs (no image is
 * valid if it exceeds capacity; the caller re-renders with a larger capacity);
 * status (device int32[2], may be NULL) = {1 if the batch fit the limits else 0,
 * number of requests rendered}.  Images are bit-identical to mgs_blend_oit of the
 * same request rendered alone.
 */
int mgs_render_batch(const mgs_request *requests, const int32_t *n_requests, int64_t max_gaussians,
                     int64_t max_tiles, uint64_t capacity, float alpha_min, float alpha_max, void *ws,
                     size_t ws_bytes, uint32_t *n_pairs, int32_t *status, void *stream);

/* ------------------------------------------------------------------------------------------
 * Contribution-based pruning (Sec. 3.3; settings in Appendix C: tau = 0.2, I_prune = 1000,
 * v = 0.6).  Per training iteration, a Gaussian whose opacity o = sigmoid(opacity_logit) lies
 * under the tau-quantile of all opacities AND whose largest scale s_max = exp(max log_scale)
 * lies under the tau-quantile of all largest scales is a pruning candidate and gains a vote.
 * At the end of a pruning interval the Gaussians with more than I_prune * v votes are removed.
 * Q_tau interpolates linearly between the sorted values at positions floor(tau (N - 1)) and
 * the next; the candidate tests "o < Q_tau(o)" and "s_max < Q_tau(s_max)" are decided exactly
 * (no rounding of Q_tau), on the stored logits and log-scales (sigmoid and exp are increasing).
 * -0.0 and +0.0 count as equal; NaN parameters are not supported.
 * ------------------------------------------------------------------------------------------ */

/* Workspace bytes of mgs_prune_vote / mgs_prune_compact for n Gaussians (n in [0, 2^31)). */
int mgs_prune_workspace(int64_t n, size_t *bytes);

/* Candidate criteria of mgs_prune_vote: Sec. 3.3 uses both; Table 4 ablates each alone. */
#define MGS_PRUNE_OPACITY 1
#define MGS_PRUNE_SCALE   2
#define MGS_PRUNE_BOTH    3

/*
 * mgs_prune_vote -- one iteration's votes.  opacity_logit [n], log_scale [3][n] (the
 * mgs_gaussians layout), device, read only.  tau in [0, 1].  criteria: MGS_PRUNE_BOTH (the
 * method), or MGS_PRUNE_OPACITY / MGS_PRUNE_SCALE alone.  votes [n] uint32, device, in/out:
 * votes[g] += 1 for every candidate g.  candidates [n] uint8 (device) receives 1 / 0 per
 * Gaussian, or is NULL.  ws: mgs_prune_workspace(n) bytes, 256-byte aligned, no initial
 * contents needed.  n = 0 enqueues nothing.  MGS_ERR_INVALID_ARG for NULL buffers, n out of
 * range, tau outside [0, 1], unknown criteria or a small workspace.  Asynchronous on `stream`.
 */
int mgs_prune_vote(const float *opacity_logit, const float *log_scale, int64_t n, double tau, int criteria,
                   void *ws, size_t ws_bytes, uint32_t *votes, uint8_t *candidates, void *stream);

/*
 * mgs_prune_compact -- the end of a pruning interval.  Gaussian g survives when votes[g] <=
 * max_votes, where max_votes = floor(I_prune * v) (votes are integers, so "more than I_prune
 * * v votes" is "more than floor(I_prune * v)").  keep_index [n] uint32 (device) receives the
 * survivors' indices in ascending order, *n_keep (device uint32) their count; entries of
 * keep_index past *n_keep are unspecified.  votes [n] is reset to zero (the next interval
 * counts from zero).  ws as for mgs_prune_vote.  Asynchronous on `stream`.
 */
int mgs_prune_compact(uint32_t *votes, int64_t n, uint32_t max_votes, void *ws, size_t ws_bytes,
                      uint32_t *keep_index, uint32_t *n_keep, void *stream);

/*
 * mgs_gather_planes -- applies a compaction to SoA attribute planes: for p < planes and
 * i < min(*n_index, n_max), dst[p * dst_stride + i] = src[p * src_stride + index[i]] (float32,
 * device).  src_stride is at least the source count (also for one plane).  index (device
 * uint32) holds indices into the source planes (each below the source count), as written by mgs_prune_compact; n_index (device uint32) its count; n_max is an upper
 * bound of that count (rows past n_max are not written), dst_stride >= n_max.  dst must not
 * overlap src.  Asynchronous on `stream`.
 */
int mgs_gather_planes(const float *src, int64_t src_stride, int planes, const uint32_t *index,
                      const uint32_t *n_index, int64_t n_max, float *dst, int64_t dst_stride, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MGS_H */
