/*
 * nis.h -- C ABI of the neural in-scattering library for AMD MI355X (gfx950).
 *
 * The library evaluates the per-shading-point hot path of the neural
 * in-scattering estimator of Fang, Feng and Cui, "A real-time rendering method
 * for high albedo anisotropic materials with multiple scattering"
 * (arXiv 2401.14051):
 *
 *   density grid --(box-filter pyramid, Sec. III.B.1)--> graded density fields
 *   --(light-direction path-density sweep, eq. 1 and eq. 15)--> graded
 *   transmittance fields --(12-layer template gather, Sec. III.B.2-4, eq. 8,
 *   eq. 24)--> per-layer lattices and squeeze statistics --(3D-CNN, Fig. 3;
 *   squeeze-excitation attention, eq. 24-26)--> 1057-entry descriptor
 *   --(backbone MLP, Fig. 6)--> log-space output y --(decode of eq. 21 plus the
 *   single-scatter term of eq. 19)--> in-scattered radiance.
 *
 * Conventions.  The medium occupies the unit cube [0,1]^3.  Density arrays are
 * float32 in [z][y][x] order, x fastest.  Extinction is sigma_t * density.
 * Light directions point TOWARDS the distant light; view directions are the
 * camera-ray directions (light reaching the camera travels along -dir).
 *
 * Errors.  Every call returns an int32_t status (NIS_OK or a negative code) and
 * never aborts or throws; nis_last_error() returns a thread-local message for
 * the last failing call on that thread.  A context is used by one host thread
 * at a time.
 *
 * Memory.  The context owns every device allocation it makes.  Host arrays
 * passed in are copied before the call returns (the caller may free them);
 * device arrays passed to the asynchronous calls are borrowed until the work
 * queued on the given stream has completed.
 *
 * Streams.  Asynchronous calls take a `hip_stream` (a hipStream_t; NULL is
 * HIP's null stream).  The work of one context is ordered across streams: the
 * work a call queues starts after the work of the context's earlier calls,
 * whatever streams those used (an event recorded at the end of each call, and
 * waited for when the next call uses another stream).  Synchronous calls
 * return after their own work completes.
 */
#ifndef NIS_H
#define NIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nis_ctx nis_ctx;

/* status codes */
#define NIS_OK 0
#define NIS_E_INVALID (-1)     /* bad argument: NULL, out of range, non-finite, malformed blob */
#define NIS_E_STATE (-2)       /* call not valid in the current state (no weights, unknown medium) */
#define NIS_E_NOMEM (-3)       /* device allocation failed or exceeded the context's budget */
#define NIS_E_DEVICE (-4)      /* a HIP runtime call failed; the HIP error text is kept */
#define NIS_E_UNSUPPORTED (-5) /* a valid request the library cannot serve (field too large) */
#define NIS_E_INTERNAL (-6)

/* network precisions (nis_set_precision) */
#define NIS_FP32 0   /* every GEMM in float32 (MFMA f32), float32 descriptor */
#define NIS_BF16 1   /* CNN and backbone GEMMs in bfloat16 x bfloat16 -> float32 */
#define NIS_FP8 2    /* backbone GEMMs in FP8-E4M3 (OCP) x E4M3 -> float32: one static
                        activation scale per layer input (from the weight blob or
                        nis_calibrate_fp8), one power-of-two weight scale per output
                        channel (the MFMA's E8M0 block scale); descriptor stored as
                        E4M3 codes; CNN in BF16 */

/* nis_set_light flags */
#define NIS_EAGER 1  /* run the transmittance sweep now rather than at the next query */

/* Template and descriptor sizes. */
#define NIS_LAYERS 12        /* 8 diffuse + 4 highlight template layers (Sec. III.B.2, III.C.2) */
#define NIS_SITES 225        /* 9 x 5 x 5 light-aligned lattice sites per layer */
#define NIS_STATS 8          /* squeeze vector per layer, eq. (24) */
#define NIS_DESCRIPTOR 1057  /* 12 x (80 + 8) + albedo */

/*
 * nis_create / nis_destroy.
 * Creates a context on HIP device `hip_device` (0-based).  The context owns
 * one HIP stream used by the synchronous calls.  destroy frees every device
 * allocation and is a no-op on NULL.
 * Errors: NIS_E_INVALID (out == NULL or bad device), NIS_E_DEVICE.
 */
int32_t nis_create(int32_t hip_device, nis_ctx **out);
int32_t nis_destroy(nis_ctx *ctx);

/*
 * nis_load_medium -- Sec. III.B.1: the density field and its down-sampled
 * graded density fields.
 * `density`: host array of n*n*n float32 in [z][y][x] order, copied before
 * return.  n must be a power of two in [1, 1024]; values finite and >= 0.
 * sigma_t >= 0 is the extinction scale (mu_t = sigma_t * density, eq. 15);
 * albedo in [0,1] (eta = mu_s / mu_t, Sec. III.C.1); g in (-1,1) is the
 * Henyey-Greenstein asymmetry (eq. 5).  Builds the 2x2x2 box-mean pyramid down
 * to 1^3 (log2(n)+1 levels) on the device.  Writes the medium handle.
 * Errors: NIS_E_INVALID, NIS_E_NOMEM, NIS_E_DEVICE.
 */
int32_t nis_load_medium(nis_ctx *ctx, const float *density, int32_t n, float sigma_t,
                        float albedo, float g, int32_t *medium_out);

/*
 * nis_rebuild_pyramid -- recomputes levels 1.. of the pyramid from the
 * resident level 0 on `hip_stream`, without any host transfer, and marks the
 * transmittance fields stale.  Asynchronous.
 */
int32_t nis_rebuild_pyramid(nis_ctx *ctx, int32_t medium, void *hip_stream);

/* Changes sigma_t, albedo and g of a loaded medium (its phase becomes the
 * single HG lobe g).  The stored path density is independent of sigma_t, so
 * no sweep is needed.  Errors as above. */
int32_t nis_set_medium_params(nis_ctx *ctx, int32_t medium, float sigma_t, float albedo, float g);

/*
 * nis_set_phase_lobes -- gives a loaded medium a multi-lobe phase (Sec. III.A,
 * eq. 6): the weighted sum of n Henyey-Greenstein lobes, weights[i] >= 0
 * summing to 1 (within 1e-5) and g[i] in (-1,1), 1 <= n <= 4; both arrays are
 * copied.  The phase enters the phase features (eq. 8), the single-scatter
 * term and, as its mean cosine sum(weights[i] g[i]), the squeeze vector
 * (eq. 24).  One lobe of weight 1 equals nis_set_medium_params' g.  Frame
 * server requests keep their own single g.  NIS_E_INVALID on a bad argument.
 */
int32_t nis_set_phase_lobes(nis_ctx *ctx, int32_t medium, int32_t n, const float *weights, const float *g);

/*
 * nis_set_volume_phase -- enable = 1 makes both factors of every site's phase
 * feature volume phases (Sec. III.A, eq. 9): the medium's phase averaged over
 * the cone under which the site, read as a ball of half the lattice spacing,
 * is seen from the point (half-angle asin(1 / (2 |o|)) for lattice offset o);
 * the centre site keeps the point phase.  The cone means are tabulated per
 * light and phase (2048 bins over the angle between w and the site direction,
 * per site, linear interpolation).  enable = 0 restores the point phases (the default).
 * NIS_E_INVALID for other values.
 */
int32_t nis_set_volume_phase(nis_ctx *ctx, int32_t medium, int32_t enable);

/*
 * nis_set_albedo_rgb -- a coloured albedo (Sec. III.C.2: one albedo per red,
 * green and blue channel, each in [0,1]; eq. 21 decodes channel c with
 * albedo_c^gamma).  albedo_rgb: host float32[3], copied.  The network runs once
 * per channel on the shared features with that channel's albedo as its input
 * entry; nis_query_rgb, nis_query_rgb_device and nis_render_rgb return the
 * three channels, and the frame server renders the medium's frames in RGB
 * (nis_frame_result.channels = 3; the albedo is read at submission).  While the
 * channels differ, the one-channel calls fail with NIS_E_STATE; three equal
 * values make the medium grey again, as does nis_set_medium_params.
 * NIS_E_INVALID for NULL or values out of range.
 */
int32_t nis_set_albedo_rgb(nis_ctx *ctx, int32_t medium, const float *albedo_rgb);

/* Frees a medium's pyramid and transmittance fields. */
int32_t nis_unload_medium(nis_ctx *ctx, int32_t medium);

/*
 * nis_set_light -- eq. (16): a distant light from direction `dir` (towards the
 * light, normalised inside; a zero or non-finite vector is NIS_E_INVALID) with
 * intensity `radiance`.  Marks the graded transmittance fields (eq. 1) stale;
 * they are recomputed by the sweep at the next query, or now with NIS_EAGER
 * (then queued on the context's own stream, ordered before later calls).
 * NIS_E_UNSUPPORTED when the light's state passes the kernels' offset limits
 * (see nis_light_footprint), NIS_E_NOMEM when it does not fit in HBM.
 */
int32_t nis_set_light(nis_ctx *ctx, int32_t medium, const float dir[3], float radiance,
                      int32_t flags);

/*
 * nis_light_footprint -- the device memory one light's state takes for an n^3
 * medium, computed on the host (no context, no GPU): the path-density pairs of
 * every level (the sheared rays of the transmittance fields of eq. 1, stored
 * as pairs along V), the light-axis density pairs, and, for a light whose
 * dominant axis is x, a transposed copy of the density pyramid.  The per-light
 * tables (under 1 MiB) are not counted.  The state is held by every medium
 * under a light, and by each frame-server slot for its frame's light.
 * `n`: the medium's edge, a power of two in [1,1024]; `dir`: towards the light,
 * any non-zero finite length.  Writes the total to *bytes_out and, when
 * `level_bytes` is not NULL, the path-density pair bytes of each level m
 * (edge n >> m) to level_bytes[m], for log2(n) + 1 levels (at most 11).
 * A finest level's path-density pairs may pass 4 GiB (a 512^3 medium under a
 * light near a cube diagonal); the kernels need each slice of them, the
 * light-axis pairs and the densities of a level below 4 GiB.
 * Errors: NIS_E_INVALID (bytes_out NULL, bad n or direction), NIS_E_UNSUPPORTED
 * (the light's layout passes those limits: every light at n = 1024), the same
 * code nis_set_light returns for that medium and light.
 */
int32_t nis_light_footprint(int32_t n, const float dir[3], int64_t *bytes_out, int64_t *level_bytes);

/*
 * nis_set_weights -- network parameters (Fig. 3, Fig. 6, eq. 24-26) as one
 * little-endian blob, copied before return:
 *   header (64 bytes): char magic[4] = "NISW"; uint32 version = 1;
 *     uint32 din = 1057; uint32 width; uint32 n_linear (>= 2); uint32 groups = 2;
 *     float lambda (graded-field coefficient base, eq. 1); float gamma (log
 *     decode exponent, eq. 21); uint32 has_fp8_scales; uint32 reserved[7] = 0;
 *   then float32 tensors, for group 0 (diffuse, layers 0-7) and group 1
 *     (highlight, layers 8-11) in turn: w1[8][1][3][3][3], b1[8],
 *     w2[16][8][3][3][3], b2[16], s1[4][16], c1[4], s2[16][4], c2[16];
 *   then for i = 0..n_linear-1: A_i[out][in], beta_i[out] with in = 1057 for
 *     i = 0 and width otherwise, out = width except 1 for the last layer;
 *   then, if has_fp8_scales, float32 activation scales (x = E4M3 code *
 *     scale, each > 0): conv1 input, conv2 input, and one per backbone layer
 *     input (2 + n_linear values);
 *   then, if has_modules (the header word after has_fp8_scales, 0 or 1), the
 *     56,706 float32 weights of the paper's backbone modules (Sec. III.C.2,
 *     Fig. 6; see nis_set_backbone): for type 0..2 (graded transmittance,
 *     density, phase), for group 0..1 (diffuse template layers 0-7, highlight
 *     8-11), for each step from layer k to k+1 of the group: S1[2][8], e1[2],
 *     S2[a][2], e2[a], F1[b][a], f1[b], F2[b][b], f2[b] with a = n_k + 2,
 *     b = n_(k+1) (n_k: the template layer's point count); then for type
 *     0..2: M[64][56], mb[64].
 * Errors: NIS_E_INVALID on a malformed blob, NIS_E_NOMEM, NIS_E_DEVICE.
 */
int32_t nis_set_weights(nis_ctx *ctx, const void *blob, size_t nbytes);

/* template kinds (nis_set_templates) */
#define NIS_TEMPLATES_LATTICE 0  /* 12 light-aligned 5x5x9 lattices with the 3D-CNN (default) */
#define NIS_TEMPLATES_PAPER 1    /* the paper's diffuse sphere and highlight cone (Sec. III.B.2) */

/*
 * nis_set_templates -- which sampling templates the context's queries and
 * renders use.  NIS_TEMPLATES_PAPER: the paper's own templates (Sec. III.B.2,
 * eq. 2-4): a diffuse sphere of 8 layers (6, 8, 12, 16, 24, 32, 48, 48
 * points; layer 0 the centre and 5 points on its sphere, layer i >= 1 a
 * shell from half its radius to its radius r_i = 2^(i-1) xi_i / (2^8 D(S_i)),
 * xi_i = 1 - 0.08 min(i, 5), D the mean nearest-neighbour distance of the
 * unit set, eq. 3) and a highlight cone of 4 layers (32, 16, 16, 8 points)
 * with its apex at the point, its axis towards the light, scaled to the
 * distance at which the light enters the medium, its layers the four equal
 * quarters of that distance.  Each layer samples the pyramid level whose
 * voxel matches its point spacing.  The network's input is then, per layer,
 * the graded transmittances, densities and phase features at its points
 * (template order) and the squeeze vector of eq. (24), zeros up to the
 * albedo entry at index 1056 (the same weight blob layout; the first layer's
 * columns 894..1055 meet zeros).  Volume phases are not available there
 * (NIS_E_UNSUPPORTED at query time).  The frame server keeps the lattices.
 * Errors: NIS_E_INVALID for an unknown kind.
 */
int32_t nis_set_templates(nis_ctx *ctx, int32_t kind);

/* backbone kinds (nis_set_backbone) */
#define NIS_BACKBONE_MLP 0    /* the template features go straight into the MLP (default) */
#define NIS_BACKBONE_PAPER 1  /* the paper's layer-by-layer modules before the MLP (Fig. 6) */

/*
 * nis_set_backbone -- NIS_BACKBONE_PAPER puts the paper's backbone modules
 * (Sec. III.C.2, Fig. 6, eq. 24-26) between the paper's templates and the
 * MLP: per feature type (graded transmittance, density, phase) and template
 * group (diffuse layers 0-7, highlight layers 8-11) one module carries the
 * features h of its current layer from layer to layer.  A step from layer k
 * fuses h with the configuration (g, alpha = acos(w.l)) into u = [h; g;
 * alpha], gates it with the attention of eq. (24)-(26) excited by the
 * layer's squeeze vector v_k (a = sigmoid(S2 ReLU(S1 v_k + e1) + e2) * u),
 * maps it to the next layer's size and fuses that layer's features x:
 * y = x + F1 a + f1, h = ReLU(F2 y + f2) + x.  Per type the two groups'
 * final states (48 + 8 values) merge, m = ReLU(M [h_D; h_H] + mb) (64
 * values), and the MLP reads [m_T; m_rho; m_phi; g; alpha] (194 entries),
 * zeros, and the albedo at index 1056.  The template features are gathered
 * in FP32 and the modules run in FP32 whatever the precision; the
 * precision sets the descriptor's format and the MLP.  Queries in this mode
 * need NIS_TEMPLATES_PAPER and weights with the module block (NIS_E_STATE
 * otherwise) and pass at most 65,536 points at a time.
 * nis_query_device_noalloc refuses it (NIS_E_UNSUPPORTED); the frame server
 * keeps the lattices.
 * Errors: NIS_E_INVALID for an unknown kind; NIS_E_STATE for
 * NIS_BACKBONE_PAPER when the current weights hold no modules.
 */
int32_t nis_set_backbone(nis_ctx *ctx, int32_t kind);

/* NIS_FP32 (default), NIS_BF16 or NIS_FP8.  FP8 needs the activation scales
 * of the weight blob's fp8 block (x = code * scale, entries > 0) or of
 * nis_calibrate_fp8; without them NIS_FP8 is NIS_E_UNSUPPORTED (here, and for
 * queries if weights without scales replace them later).  The scales are
 * static, so a point's result does not depend on its batch.  The blob's two
 * CNN-input scales are kept and unused (the CNN runs in BF16).
 * Errors: NIS_E_INVALID for an unknown precision, NIS_E_UNSUPPORTED. */
int32_t nis_set_precision(nis_ctx *ctx, int32_t precision);

/*
 * nis_calibrate_fp8 -- the static activation scales of the FP8 backbone
 * (per-layer absmax scaling of E4M3, Sec. III.C.2's network in FP8): runs the
 * FP32 path over n representative points (device arrays as nis_query_device)
 * of `medium` under its light, records the largest |input| of every backbone
 * layer (the descriptor, then each hidden activation), and sets each layer
 * input's scale to 2 max|x| / 448 (codes saturate at 448, so a factor of two
 * above the calibration range is kept).  Replaces the blob's scales and
 * repacks the FP8 weights.  Synchronous on `hip_stream`.
 * Errors: NIS_E_INVALID, NIS_E_STATE (no weights, no light, server running).
 */
int32_t nis_calibrate_fp8(nis_ctx *ctx, int32_t medium, const float *d_points,
                          const float *d_view_dirs, int64_t n, void *hip_stream);

/*
 * nis_query -- in-scattered radiance at shading points (Sec. III.C.2 output
 * layer; eq. 19, eq. 21):  L = I * (f(w.l) T(p) + albedo^gamma expm1(y)), f the
 * medium's phase (HG, or the HG lobes of nis_set_phase_lobes).
 * `points`: host float32 [n][3] in unit-cube coordinates (may lie outside);
 * `view_dirs`: host float32 [n][3], normalised inside; `radiance_out`: host
 * float32 [n].  Synchronous.  Errors: NIS_E_INVALID (n <= 0, NULL, non-finite
 * input, zero direction), NIS_E_STATE (unknown medium, no light, no weights, a
 * coloured albedo).
 */
int32_t nis_query(nis_ctx *ctx, int32_t medium, const float *points, const float *view_dirs,
                  int64_t n, float *radiance_out);

/*
 * nis_query_rgb -- as nis_query with one radiance per colour channel:
 * radiance_out is host float32 [n][3], channel c computed with albedo_c
 * (nis_set_albedo_rgb; a grey medium gives three copies of nis_query's
 * result).  The features are computed once and the backbone runs three times.
 */
int32_t nis_query_rgb(nis_ctx *ctx, int32_t medium, const float *points, const float *view_dirs,
                      int64_t n, float *radiance_out);

/* One query of a batch (nis_query_batch): n points of `medium` under its
 * light, device arrays as for nis_query_device. */
typedef struct nis_query_item {
    int32_t medium;
    int32_t reserved;           /* 0 */
    const float *d_points;      /* [n][3] */
    const float *d_view_dirs;   /* [n][3] */
    int64_t n;                  /* >= 0 */
    float *d_radiance_out;      /* [n] */
} nis_query_item;

/*
 * nis_query_batch -- `count` (1..64) queries, possibly over different media
 * each under its own light and phase, as one gather launch and one backbone
 * launch (Sec. III.C.2: the network is evaluated for many template positions
 * in parallel; the paper's own use queries 4129 template centres per
 * medium).  Each query's radiance equals, bit for bit, what
 * nis_query_device gives it alone.  The light fields and site tables of each
 * medium are brought up to date first, then the gather reads each query's
 * medium from a table (its workgroups a contiguous range of the grid), the
 * backbone runs once over all rows, and each query's decode writes its
 * output.  At most 2^21 points in all; the lattice templates and a grey
 * albedo only.  Queued on `hip_stream` like nis_query_device.
 * Errors: NIS_E_INVALID (count, an item, more than 2^21 points),
 * NIS_E_STATE (no weights, unknown medium, a coloured medium),
 * NIS_E_UNSUPPORTED (the paper's templates; FP8 without scales).
 */
int32_t nis_query_batch(nis_ctx *ctx, const nis_query_item *items, int32_t count, void *hip_stream);

/* nis_query_rgb_device -- nis_query_rgb on device arrays (d_radiance_out
 * float32 [n][3]), queued on `hip_stream` as nis_query_device. */
int32_t nis_query_rgb_device(nis_ctx *ctx, int32_t medium, const float *d_points,
                             const float *d_view_dirs, int64_t n, float *d_radiance_out,
                             void *hip_stream);

/*
 * nis_query_device -- as nis_query on device arrays, queued on `hip_stream`
 * and returning before the work completes.  Inputs are not validated
 * element-wise.  Scratch memory is owned by the context and reused by its
 * next call (which the ordering above makes safe).
 */
int32_t nis_query_device(nis_ctx *ctx, int32_t medium, const float *d_points,
                         const float *d_view_dirs, int64_t n, float *d_radiance_out,
                         void *hip_stream);

/*
 * nis_query_device_noalloc -- nis_query_device for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same computation and the same result,
 * bit for bit, but the call allocates nothing.  Its scratch (descriptor rows and
 * single-scatter terms of one pass) is a fixed array of
 * device memory inside the library, about 36 MB, of which each GPU the library
 * runs on holds its own copy until the process ends; no part of it has to
 * start at zero.  Every call on one GPU shares that GPU's copy, which keeps
 * the last call's contents: calls whose work overlaps on one GPU (other
 * streams, other contexts, other host threads) race, and the caller must
 * order them.  Limits: 1 <= n <= NIS_NOALLOC_MAX_POINTS points per call
 * (NIS_E_INVALID beyond); the medium's light must have been set (its fields
 * and tables are allocated by nis_set_light, and by nis_set_volume_phase for
 * volume phases), else NIS_E_STATE.  Arguments, layouts, ownership, ordering
 * and other errors as nis_query_device.
 */
#define NIS_NOALLOC_MAX_POINTS 8192
int32_t nis_query_device_noalloc(nis_ctx *ctx, int32_t medium, const float *d_points,
                                 const float *d_view_dirs, int64_t n, float *d_radiance_out,
                                 void *hip_stream);

/* ---- frames --------------------------------------------------------------- */

/*
 * A camera.  vfov_deg in (0,180): pinhole at `eye` looking at `target` with
 * `up` fixing the roll; the vertical field of view is vfov_deg and the
 * horizontal one follows from width / height.  Pixel (col, row), row 0 at the
 * top, is index row * width + col; its ray passes through the pixel centre.
 * vfov_deg == 0: orthographic rays along -z through the pixel centres of the
 * unit square at height ortho_z (x = (col + 0.5) / width, y = (row + 0.5) /
 * height).  At most 2^28 pixels.
 */
typedef struct nis_camera {
    double eye[3];
    double target[3];
    double up[3];
    double vfov_deg;
    double ortho_z;
    int32_t width;
    int32_t height;
} nis_camera;

/*
 * nis_frame_points -- the shading points of a frame: for each pixel's ray,
 * the first real collision inside the unit cube found by delta tracking on the
 * finest density level read as piecewise constant per voxel (majorant
 * sigma_t * max density; free flights -log(1-u)/majorant; acceptance with
 * probability sigma_t * rho / majorant; u from the SplitMix64 hash
 * mix(mix(mix(seed) ^ pixel) ^ draw), top 53 bits, draw 2i for the i-th flight
 * and 2i+1 for its acceptance; at most 100000 flights per ray).  Writes the
 * collisions compacted in pixel order: d_points and d_dirs float32 [P][3]
 * (ray direction, unit), d_pixel int32 [P], and P to d_count (one int32).  All
 * four are device arrays sized for width*height entries, borrowed until the
 * work queued on `hip_stream` completes.  Asynchronous.
 * Errors: NIS_E_INVALID (NULL output, bad camera), NIS_E_STATE.
 */
int32_t nis_frame_points(nis_ctx *ctx, int32_t medium, const nis_camera *camera, uint64_t seed,
                         float *d_points, float *d_dirs, int32_t *d_pixel, int32_t *d_count,
                         void *hip_stream);

/*
 * nis_render -- one frame (eq. 19 at every collision): the points of
 * nis_frame_points queried at the context's precision, and
 * d_image[row * width + col] = albedo * L at a collision, 0 where the ray
 * leaves the medium.  d_image is a device float32 array of width*height
 * entries.  Queued on `hip_stream` with no host synchronisation: the query
 * reads the collision count from device memory.  Errors as nis_query_device.
 */
int32_t nis_render(nis_ctx *ctx, int32_t medium, const nis_camera *camera, uint64_t seed,
                   float *d_image, void *hip_stream);

/*
 * nis_render_rgb -- nis_render with a coloured albedo: d_image is a device
 * float32 array [width*height][3], d_image[3 * pixel + c] = albedo_c * L_c at a
 * collision and 0 elsewhere, L_c the radiance of nis_query_rgb.  The frame
 * points are the same as nis_render's (they do not depend on the albedo).
 */
int32_t nis_render_rgb(nis_ctx *ctx, int32_t medium, const nis_camera *camera, uint64_t seed,
                       float *d_image, void *hip_stream);

/* ---- frame server -------------------------------------------------------------
 *
 * A scheduler thread owned by the context takes frame requests from any
 * number of host threads and keeps up to max_inflight of them on the device at
 * once, each on its own stream with its own light fields and workspace,
 * admitting the oldest queued request as soon as a stream is free and the
 * device memory it needs fits the budget (first come, first served).  A
 * frame's image does not depend on what else is in flight.  The server calls
 * are thread-safe.  While a server runs, nis_set_weights, nis_unload_medium and
 * nis_rebuild_pyramid return NIS_E_STATE; other calls stay valid.
 */

#define NIS_QUEUED 1    /* nis_frame_result.status: waiting for admission */
#define NIS_RUNNING 2   /* on the device */

typedef struct nis_server_cfg {
    uint64_t hbm_budget_bytes;  /* device memory the server may hold: per-stream light
                                   fields and workspaces plus every unreleased image */
    int32_t precision;          /* NIS_FP32, NIS_BF16 or NIS_FP8 */
    int32_t max_inflight;       /* frames on the device at once, 1..16 */
    int32_t batch_gather;       /* 1: small grey frames (<= 2^18 pixels) admitted together
                                   share one gather launch (results unchanged); 0: off */
    int32_t reserved;           /* 0 */
} nis_server_cfg;

typedef struct nis_frame_req {
    int32_t medium;
    nis_camera camera;
    float light_dir[3];         /* towards the light, normalised inside */
    float radiance;             /* light intensity I */
    float g;                    /* HG asymmetry of this frame, in (-1,1) */
    uint64_t seed;              /* delta-tracking seed */
} nis_frame_req;

typedef struct nis_frame_result {
    int32_t status;             /* NIS_QUEUED, NIS_RUNNING, NIS_OK (done) or a negative error */
    int32_t width, height;
    int32_t channels;           /* 1, or 3 for a medium with a coloured albedo (nis_set_albedo_rgb) */
    int64_t n_points;           /* collisions shaded (valid when done) */
    const float *d_image;       /* device [height][width][channels] float32, valid until nis_release */
    double t_submit, t_start, t_done;   /* seconds since nis_server_start (host steady clock):
                                           submitted, admitted, completion observed */
} nis_frame_result;

/* Device memory the server holds while it runs the frame `req` at `precision`:
 * the query workspace, the per-pixel frame buffers, the light's path-density
 * fields and site tables, and the image.  Needs no server. */
int32_t nis_frame_memory(nis_ctx *ctx, const nis_frame_req *req, int32_t precision,
                         uint64_t *bytes);

/* Starts the server.  NIS_E_STATE if one runs or no weights are set;
 * NIS_E_INVALID for a bad configuration. */
int32_t nis_server_start(nis_ctx *ctx, const nis_server_cfg *cfg);

/* Queues a frame and writes its id.  The medium's sigma_t and albedo are read
 * now.  NIS_E_NOMEM if the frame alone needs more than the whole budget;
 * NIS_E_INVALID / NIS_E_STATE for bad requests or no server. */
int32_t nis_submit_frame(nis_ctx *ctx, const nis_frame_req *req, uint64_t *id);

/* Current state of a frame; never blocks.  NIS_E_INVALID for an unknown id. */
int32_t nis_poll(nis_ctx *ctx, uint64_t id, nis_frame_result *out);

/* As nis_poll, but blocks until the frame is done or failed. */
int32_t nis_wait(nis_ctx *ctx, uint64_t id, nis_frame_result *out);

/* Returns a finished frame's image memory to the server.  NIS_E_STATE while
 * the frame is queued or running. */
int32_t nis_release(nis_ctx *ctx, uint64_t id);

/* Waits for the frames on the device, drops queued ones, frees every server
 * allocation (unreleased images included) and stops the thread.  NIS_E_STATE if
 * no server runs. */
int32_t nis_server_stop(nis_ctx *ctx);

/* Thread-local message of the last failing call ("" if none). */
const char *nis_last_error(void);

/* ---- stage access, for testing and profiling --------------------------- */

/*
 * nis_profile -- when enable != 0, every kernel the context launches is
 * bracketed by HIP events recorded on the stream it runs on, and durations
 * are accumulated per kernel name ("pyramid", "sweep", "site_tables",
 * "features", "backbone").  Synchronizes the device and clears earlier records.
 */
int32_t nis_profile(nis_ctx *ctx, int32_t enable);

/* Writes one line "name launches total_ms" per kernel into buf (synchronizes
 * on the recorded events).  NIS_E_INVALID if buf is too small. */
int32_t nis_profile_report(nis_ctx *ctx, char *buf, size_t capacity);

/* Number of pyramid levels and the float count of all levels together. */
int32_t nis_medium_info(nis_ctx *ctx, int32_t medium, int32_t *levels, int64_t *pyramid_floats);

/* Copies all pyramid levels (level 0 first, each n_m^3 [z][y][x]) to host. */
int32_t nis_debug_pyramid(nis_ctx *ctx, int32_t medium, float *out, int64_t capacity);

/*
 * Runs the sweep if stale and copies level `level`'s path density
 * D[J][V][U] to host.  dims[0..4] = U_lo, U_hi, V_lo, V_hi, n_J.  Pass
 * out = NULL to query dims only.
 */
int32_t nis_debug_path_density(nis_ctx *ctx, int32_t medium, int32_t level, float *out,
                               int64_t capacity, int32_t dims[5]);

/*
 * Runs the sweep if stale and copies level `level`'s path-density pairs to
 * host: [J][V' = 0..n_V][U] float pairs (D(V'-1), D(V')) with V' - 1 and V'
 * clamped into the level's ray range: the layout the gather reads, without
 * its padding rays along U (the same values as D, rearranged; eq. 1).
 * capacity counts floats and must be at least 2 n_J (n_V + 1) n_U, with the
 * dims of nis_debug_path_density.
 */
int32_t nis_debug_path_pairs(nis_ctx *ctx, int32_t medium, int32_t level, float *out, int64_t capacity);

/*
 * Gather stage on device arrays (synchronous): tbar/rho [n][12][225],
 * phi [n][225], stats [n][12][8], tp [n] (transmittance to the light),
 * f0 [n] (single-scatter term f(w.l) T(p)).  Any output may be NULL.
 */
int32_t nis_debug_features(nis_ctx *ctx, int32_t medium, const float *d_points,
                           const float *d_view_dirs, int64_t n, float *d_tbar, float *d_rho,
                           float *d_phi, float *d_stats, float *d_tp, float *d_f0);

/*
 * Gather stage at the paper's templates (whatever nis_set_templates holds;
 * synchronous): tbar/rho/phi [n][266] in template order (the 8 diffuse
 * layers, then the 4 highlight layers), stats [n][12][8] (eq. 24), f0 [n]
 * (may be NULL).  The other arrays are required.
 */
int32_t nis_debug_template_features(nis_ctx *ctx, int32_t medium, const float *d_points,
                                    const float *d_view_dirs, int64_t n, float *d_tbar,
                                    float *d_rho, float *d_phi, float *d_stats, float *d_f0);

/*
 * Descriptor and network output on device arrays (synchronous), at the
 * current precision: desc [n][1057] float32 (the values the backbone reads),
 * y [n].  Either may be NULL.
 */
int32_t nis_debug_network(nis_ctx *ctx, int32_t medium, const float *d_points,
                          const float *d_view_dirs, int64_t n, float *d_desc, float *d_y);

#ifdef __cplusplus
}
#endif

#endif /* NIS_H */
