/* tide.h -- C ABI of the MI355X (gfx950) training hot path of out-of-core
 * 3D Gaussian Splatting (TideGS, arXiv 2605.20150).
 *
 * The paper keeps the standard 3DGS forward/backward on the resident
 * Gaussians (Sec. 3.3, "Level 2") and adds a block tier around it (Sec. 3.3
 * to 3.5, Alg. 1).  This header exposes both halves:
 *
 *   per iteration, on the GPU          tide_preprocess -> tide_bin_sort ->
 *                                      tide_render_fwd -> tide_loss ->
 *                                      tide_render_bwd -> tide_adam_sparse
 *   around it, on the host             tide_cull_blocks, tide_stream_delta,
 *                                      tide_ensure_resident, ...
 *   learned prefetch predictor         tide_mlp_*
 *
 * Conventions shared by every call
 *   - Device memory is owned by the caller.  Pointers documented as "device"
 *     must be device (HBM) pointers; "host" pointers are ordinary memory.
 *     The library never allocates device memory on the per-iteration path;
 *     calls that need scratch take a caller workspace (ws, ws_bytes) and
 *     report the size they need.  Device buffers and workspaces must be at
 *     least 8-byte aligned (f64 data: 8; records of four-byte values are
 *     moved as unaligned 16-byte pieces, which need 4); 256-byte alignment,
 *     what hipMalloc and torch give, lets the scans, histograms and range
 *     pass of tide_bin_sort use 16-byte accesses (they fall back to
 *     one-element accesses otherwise).
 *   - Device work is enqueued on the HIP stream passed as `stream`
 *     (a hipStream_t; NULL = the default stream) and is asynchronous unless a
 *     call says it blocks.
 *   - Every call returns a tide_status; nothing throws across the ABI.
 *     Arguments are validated on the host before anything is launched.
 *     tide_last_error() returns a thread-local message for the last failure.
 *   - Parameter rows have TIDE_D = 59 columns: mean(3), log-scale(3),
 *     quaternion w,x,y,z (4), opacity logit (1), SH degree-3 coefficients
 *     16 x (r,g,b) coefficient-major (48).  (Sec. 2, D = 59.)
 *   - dtype TIDE_F32 is the training path; TIDE_F64 is the same kernels
 *     instantiated in double precision for gradient checks.
 */
#ifndef TIDE_H
#define TIDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tide_status;
#define TIDE_OK 0
#define TIDE_EINVAL (-1)     /* bad argument (null, misaligned, size, dtype) */
#define TIDE_ECAPACITY (-2)  /* a caller buffer is too small; the call says which size it needs */
#define TIDE_EHIP (-3)       /* a HIP runtime call failed */
#define TIDE_EIO (-4)        /* file I/O failed (block store) */
#define TIDE_ESTATE (-5)     /* call out of order / object in the wrong state */

#define TIDE_F32 0
#define TIDE_F64 1
#define TIDE_D 59
#define TIDE_TILE 16
#define TIDE_MAX_CAMS 8

const char* tide_last_error(void);
int32_t tide_abi_version(void);

/* ------------------------------------------------------------------------
 * Cameras (host structs).  World-to-camera p_cam = R p_world + t, R
 * row-major, OpenCV axes (x right, y down, z forward).  Pixel (i, j) is
 * sampled at (i + 0.5, j + 0.5).  Tiles are 16 x 16, ceil(W/16) x ceil(H/16).
 * z_near / z_far cull a Gaussian whose camera depth is <= z_near or > z_far;
 * the same planes bound the block frustum test of tide_cull_blocks.
 * ---------------------------------------------------------------------- */
typedef struct {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
  double z_near, z_far;
} tide_camera;

/* ------------------------------------------------------------------------
 * Resident parameter pool (Sec. 3.3, Eq. block_def: Block(k) = rows
 * [kB, (k+1)B) of the table).  GPU memory is a set of block slots, stored
 * block-SoA: X[slot][col][row], so every column of a block is contiguous.
 *   params, exp_avg, exp_avg_sq  device, [n_slots][59][block_rows], dtype
 *   step        device u32 [n_slots][block_rows]: Adam steps taken per row
 *   slot_block  device i32 [n_slots]: global block id held by the slot, -1 free
 *   slot_rows   device i32 [n_slots]: valid rows in the slot (the last block
 *               of the table may be partial)
 *   order       device i32 [n_order]: slots to render, in ascending block id.
 *               Processing index pidx = k * block_rows + row for order[k];
 *               global id gid = slot_block[order[k]] * block_rows + row, so
 *               pidx order is global-id order wherever the blocks sit.
 * ---------------------------------------------------------------------- */
typedef struct {
  void* params;
  void* exp_avg;
  void* exp_avg_sq;
  uint32_t* step;
  const int32_t* slot_block;
  const int32_t* slot_rows;
  const int32_t* order;
  int32_t n_slots;
  int32_t block_rows;
  int32_t n_order;
  int32_t dtype;
} tide_pool;

/* ------------------------------------------------------------------------
 * Per (camera, Gaussian) projection records written by tide_preprocess;
 * all device, caller allocated, n_pidx = n_order * block_rows.
 *   rec     [n_cams][n_pidx][12] dtype: u, v, conic A, B, C, opacity,
 *           r, g, b, depth, footprint radius (px), 0
 *           (valid where tiles_touched > 0)
 *   depth   f32 [n_cams][n_pidx] camera-space depth (the sort key)
 *   rect    u32 [n_cams][n_pidx][2]: x0 | y0 << 16, x1 | y1 << 16 (tiles,
 *           half-open)
 *   tiles_touched u32 [n_cams][n_pidx]: 0 = culled for that camera
 *   active  u32 [n_pidx]: 1 if kept by any camera of the batch
 *   act_idx u32 [n_pidx]: exclusive prefix sum of active (compact row index)
 *   n_active device u32 [1]: number of active rows
 * ---------------------------------------------------------------------- */
typedef struct {
  void* rec;
  float* depth;
  uint32_t* rect;
  uint32_t* tiles_touched;
  uint32_t* active;
  uint32_t* act_idx;
  uint32_t* n_active;
  int64_t n_pidx;
  int32_t n_cams;
  int32_t dtype;
} tide_proj;

/* Bytes of device workspace tide_preprocess needs (for the active scan). */
size_t tide_preprocess_ws_bytes(int64_t n_pidx);

/* Projection, culling, EWA footprint, tile rectangle and SH-degree-3 colour
 * of every resident Gaussian for each of the n_cams cameras (standard 3DGS
 * preprocessing, Sec. 3.3 Level 2), plus the active set I_t (Sec. 2: Gaussians
 * kept by some camera of the batch) and its compaction in pidx order.
 * cams: host array of n_cams (1..TIDE_MAX_CAMS). Asynchronous. */
tide_status tide_preprocess(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                            tide_proj* out, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of tide_preprocess, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, checks and results as
 * tide_preprocess, without the workspace: the active scan's scratch (its
 * per-4096-pidx block sums and total) is a static device array of
 * TIDE_PREPROCESS_NOALLOC_SCRATCH bytes, one per GPU, whose address is looked
 * up on the first call on each device (hipGetSymbolAddress) and which is held
 * until the process ends.  The call allocates nothing, host or device.
 *   n_pidx above TIDE_PREPROCESS_NOALLOC_MAX_PIDX -> TIDE_ECAPACITY, before
 *   any device work (use tide_preprocess with a workspace instead).
 * Every call on a GPU shares that GPU's scratch and leaves its contents there;
 * nothing in it needs to start at zero (each call writes what it reads).
 * Calls that overlap on one GPU (two streams, two host threads) race on it:
 * the caller serialises them. */
#define TIDE_PREPROCESS_NOALLOC_SCRATCH 262144
#define TIDE_PREPROCESS_NOALLOC_MAX_PIDX 134086656 /* 32736 scan blocks of 4096 */
tide_status tide_preprocess_noalloc(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                    tide_proj* out, void* stream);

/* ------------------------------------------------------------------------
 * Tile binning and depth sort, the tile stage of the standard 3DGS
 * rasterization pipeline that the paper runs unchanged on the resident
 * visible blocks (Sec. 3.3, Level 2; Sec. 3.2, Stage 3).  Every kept
 * (camera, Gaussian) pair is
 * duplicated once per covered tile and the instances are ordered by
 * (camera, tile, depth, pidx): first the visible pairs are sorted stably by
 * depth (LSD radix, 8-bit digits, one kernel per digit whose tiles find
 * their offsets by decoupled look-back), then the instances, emitted in that
 * depth order, are sorted stably by global tile id (camera * tiles + tile).
 * Results live in the caller's workspace; tide_bins points into it.
 * ---------------------------------------------------------------------- */
typedef struct {
  /* outputs (device pointers into ws) */
  const uint32_t* vis_rec;     /* [n_vis] record index c*n_pidx+pidx, depth order */
  const uint32_t* inst_off;    /* [n_vis+1] first instance of each vis entry */
  const uint32_t* inst_e;      /* [n_inst] emission index of the j-th sorted instance */
  const uint32_t* inst_rec;    /* [n_inst] record index of emission index e */
  const uint32_t* ranges;      /* [n_cams*n_tiles][2] sorted-instance [start, end) */
  const uint32_t* tile_order;  /* [n_cams*n_tiles] global tile ids by descending list length
                                  on a log scale, 16 steps per octave of length + 1 (lengths
                                  >= 2^16 together; ties in tile order): the compositing
                                  launch order */
  unsigned long long* tile_visits;  /* [2][n_cams*n_tiles] scratch in ws: per-tile visit
                                  counts that tide_render_fwd writes and sums per view */
  int64_t n_vis;
  int64_t n_inst;
  int32_t n_cams;
  int32_t tiles_x, tiles_y;
  int64_t n_pidx;
  /* set on TIDE_ECAPACITY: the workspace bytes this call needs */
  size_t ws_required;
} tide_bins;

/* Bytes of workspace for given sizes (n_inst_cap = instance capacity). */
size_t tide_bin_sort_ws_bytes(int32_t n_cams, int64_t n_pidx, int32_t tiles_x, int32_t tiles_y,
                              int64_t n_inst_cap);

/* Blocks once, until the visible-pair and instance counts have reached the
 * host; the rest of the binning is queued before that wait (sized by the
 * workspace's instance capacity, reading the counts on the device), so the
 * GPU keeps working meanwhile.  The counts go through a pinned host slot
 * allocated on the first call, one per device, which concurrent calls on a
 * device take in turn.  On TIDE_ECAPACITY, out->ws_required holds the size
 * to retry with (the projection records are unchanged and may be reused).
 * TIDE_EHIP also reports a depth-sort tile whose look-back wait exceeded
 * its poll limit (a guard that ends the wait instead of hanging; it does not
 * fire while workgroups start in index order): the lists of that call are
 * then invalid and its tile ranges empty. */
tide_status tide_bin_sort(const tide_proj* proj, int32_t tiles_x, int32_t tiles_y, void* ws,
                          size_t ws_bytes, tide_bins* out, void* stream);

/* ------------------------------------------------------------------------
 * Front-to-back alpha compositing per 16x16 tile (standard 3DGS forward;
 * Sec. 3.2 Stage 3).  For each pixel: alpha = min(0.99, opacity * exp(power)),
 * entries with power > 0 or alpha < 1/255 are skipped, and the walk stops
 * before an entry that would take the transmittance below 1e-4.
 *   image   device dtype [n_cams][3][H][W]; out = colour + T * bg
 *   t_final device dtype [n_cams][H][W]
 *   last    device u32 [n_cams][H][W]: 1 + position (in the tile list) of
 *           the last contributing entry, 0 if none
 *   visits  device u64 [2][n_cams]: row 0 the entries evaluated, summed
 *           over pixels (the entry that stops a pixel is counted); row 1
 *           the entries the backward walks, summed over pixels (the sum of
 *           last); accumulated, so zero them first.
 * bg: host float[3]. All cameras share W = width, H = height. */
typedef struct {
  void* image;
  void* t_final;
  uint32_t* last;
  unsigned long long* visits;
  int32_t width, height;
} tide_frame;

tide_status tide_render_fwd(const tide_proj* proj, const tide_bins* bins, const float* bg,
                            tide_frame* frame, void* stream);

/* ------------------------------------------------------------------------
 * Photometric loss 0.8 L1 + 0.2 (1 - SSIM) averaged over views (the paper's
 * per-view photometric loss f_i, Appendix A; weights and SSIM as standard in
 * 3DGS: 11x11 Gaussian window, sigma 1.5, zero padding, C1 = 1e-4,
 * C2 = 9e-4).
 *   image, target  device dtype [n_views][3][H][W]
 *   d_loss         device double [1] (written)
 *   d_dimage       device dtype [n_views][3][H][W]: dL/dimage (written)
 * Needs tide_loss_ws_bytes() of workspace. */
size_t tide_loss_ws_bytes(int32_t n_views, int32_t height, int32_t width, int32_t dtype);
tide_status tide_loss(const void* image, const void* target, int32_t n_views, int32_t height,
                      int32_t width, int32_t dtype, double* d_loss, void* d_dimage, void* ws,
                      size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Backward of the rasterizer, the standard 3DGS backward that the paper runs
 * on the resident blocks (Sec. 3.2, Stage 3; Sec. 3.3, Level 2: only the
 * contributing set I_t receives non-zero gradients, so the gradient is kept
 * compact over the active rows): the compositing adjoint per tile (reverse walk
 * from each pixel's last contributor), a fixed-order sum of per-instance
 * 2-D gradients per (camera, Gaussian), then the adjoint of projection,
 * EWA, activations and SH, summed over cameras in order.  Deterministic:
 * no floating-point atomics.
 *   d_dimage  device dtype [n_cams][3][H][W]
 *   grad      device dtype [59][grad_ld]: column-major compact gradient,
 *             row a = the a-th active pidx (act_idx); grad_ld >= n_pidx
 *   ws        tide_render_bwd_ws_bytes(bins) bytes
 * ---------------------------------------------------------------------- */
size_t tide_render_bwd_ws_bytes(const tide_bins* bins, int32_t dtype);
tide_status tide_render_bwd(const tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                            const tide_proj* proj, const tide_bins* bins, const tide_frame* frame,
                            const float* bg, const void* d_dimage, void* grad, int64_t grad_ld,
                            void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Masked (sparse) Adam on the active rows only (Appendix A, masked update
 * equation): for each active row, step += 1, then per column j
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr[j] * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * Inactive rows are not touched.  Each updated block is marked dirty
 * (Sec. 3.5, "GPU-side training on the resident set") and its bounding
 * sphere radius is raised to cover the updated rows (Sec. 3.3: bounds are
 * refreshed conservatively as centres move):
 *   r_k = max(r_k, |mu_i - c_k| + 3 kappa max(exp(log-scale_i))).
 *   spheres  device f32 [n_blocks][4] (cx, cy, cz, r), indexed by global block
 *   dirty    device u8 [n_blocks]
 * Either may be NULL to skip that bookkeeping.
 * ---------------------------------------------------------------------- */
typedef struct {
  float lr[TIDE_D];
  float beta1, beta2, eps;
  float kappa;
} tide_adam_cfg;

size_t tide_adam_ws_bytes(int64_t n_pidx);
/* ws: tide_adam_ws_bytes(proj->n_pidx) bytes of device scratch, 16-byte
 * aligned (the double-precision per-row bias corrections of the TIDE_F64
 * update). */
tide_status tide_adam_sparse(tide_pool* pool, const tide_proj* proj, const void* grad,
                             int64_t grad_ld, const tide_adam_cfg* cfg, float* spheres,
                             uint8_t* dirty, int64_t n_blocks, void* ws, size_t ws_bytes,
                             void* stream);

/* ------------------------------------------------------------------------
 * tide_render_bwd followed by tide_adam_sparse without the gradient in
 * between: the training step's backward and optimiser (Sec. 3.2, Stage 3;
 * Appendix A, masked update equation).  The last backward stage hands each
 * active row's 59 gradient values straight to that row's masked Adam update
 * (step += 1, moments, parameters), then the dirty marks and the sphere
 * refresh run as in tide_adam_sparse.  The pool's parameters, moments and
 * step counters end bit-identical to tide_render_bwd then tide_adam_sparse
 * on the same inputs; no gradient is stored.
 *   arguments  as tide_render_bwd (without grad) and tide_adam_sparse
 *              (without grad and its workspace)
 *   ws         tide_render_bwd_ws_bytes(bins, dtype) bytes
 * Errors as the two calls it replaces; nothing is launched on an argument
 * error.
 * ---------------------------------------------------------------------- */
tide_status tide_render_bwd_adam(tide_pool* pool, const tide_camera* cams, int32_t n_cams,
                                 const tide_proj* proj, const tide_bins* bins,
                                 const tide_frame* frame, const float* bg, const void* d_dimage,
                                 const tide_adam_cfg* cfg, float* spheres, uint8_t* dirty,
                                 int64_t n_blocks, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Out-of-core block tier (Sec. 3.3 to 3.5; Alg. 1).  A host object owns the
 * SSD log store (an immutable base segment plus append-only patch segments
 * and Index[k] = (file_id, offset, size, version), Sec. 3.4), a host LRU
 * block cache with dirty bits (pinned memory), I/O threads, and the GPU slot
 * table of the caller's tide_pool.  Device memory stays the caller's: the
 * pool arrays, the pool's slot_block / slot_rows / order arrays (written by
 * the tier) and the bounding spheres.
 *
 * A block record is the block's parameters, Adam moments and steps in the
 * pool's slot layout: params[59][B], m[59][B], v[59][B] (f32), step[B] (u32).
 *
 * Per iteration t (the paper's stages 1 to 4):
 *   tide_residency_sync_bounds   wait for the last iteration's sphere / dirty
 *                                read-back (bounds only grow, Sec. 3.3)
 *   tide_cull_blocks             K_t per camera (Level 1, Eq. Kt_def)
 *   tide_ensure_resident         make every block of K_t resident; blocks not
 *                                yet transferred are fetched synchronously
 *                                (the time spent waiting is the stall)
 *   ... compute of iteration t on the compute stream ...
 *   tide_cull_blocks             K_{t+1} per camera of the next batch
 *   tide_stream_delta            Alg. 1: R_{t+1}, S+, S-; enqueues the
 *                                transfers on the side stream behind the
 *                                compute of iteration t
 *   tide_residency_end_iteration records the compute event and reads the
 *                                refreshed spheres and dirty flags back
 * ---------------------------------------------------------------------- */
typedef struct tide_residency tide_residency;

#define TIDE_TIER_HOST_POOL 1   /* pool / spheres / dirty are host memory (CPU-only runs) */
#define TIDE_TIER_ODIRECT 2     /* O_DIRECT reads and writes of the segment files */
/* Ablations of the paper's techniques (Sec. 4.4, the ablation table):
 * NO_TIDE     no differential streaming: R_{t+1} = K_{t+1}, every block of
 *             K_{t+1} is transferred again and every resident block leaves
 *             (written back when dirty or in use);
 * NO_OVERLAP  transfers serialised with compute: tide_stream_delta waits for
 *             the current compute, then for its reads and copies, before it
 *             returns, and tide_prefetch_hint waits for its reads (the
 *             blocked time is counted as stall).
 * Neither changes which blocks a render sees, so results are unchanged. */
#define TIDE_TIER_NO_TIDE 4
#define TIDE_TIER_NO_OVERLAP 8
/* The paper's default placement and budget (Sec. 3.5), which give up the
 * bit-identity with all-resident training:
 * COLD_RESTART  Adam moments and steps live only while a block is resident:
 *               an admitted block gets its parameters and zero m, v and step;
 *               an evicted block sends back its parameters only.  The moments
 *               held in the segment files are neither read nor maintained
 *               (a store written this way is reopened with the same flag).
 * BOUNDED       the budget C binds: tide_ensure_resident renders R_t and K_t's
 *               intersection and fetches nothing (the blocks of K_t outside
 *               R_t are counted in `skipped`).  The first batch is made
 *               resident by a tide_stream_delta from the empty set. */
#define TIDE_TIER_COLD_RESTART 16
#define TIDE_TIER_BOUNDED 32

typedef struct {
  const char* dir;            /* directory of the segment files (created if missing) */
  int64_t n_rows;             /* N, rows of the whole table */
  int32_t block_rows;         /* B */
  int32_t capacity;           /* C: blocks Alg. 1 may keep resident (<= pool n_slots) */
  int64_t host_cache_blocks;  /* host LRU capacity in blocks */
  int32_t io_threads;         /* SSD worker threads (>= 1) */
  int32_t flags;              /* TIDE_TIER_* */
  double lambda_;             /* s(k) = lambda 1[k in K_{t+1}] + (1 - lambda) Recency(k) */
  double gamma;               /* Recency(k) = gamma^age */
  double kappa;               /* footprint stretch bound used by the bounds */
} tide_store_cfg;

typedef struct {
  int64_t iterations;
  int64_t blocks_in, blocks_out;          /* S+ and S- totals */
  int64_t readmissions;                   /* S+ blocks that had been resident before */
  int64_t h2d_bytes, d2h_bytes;           /* PCIe traffic of block records */
  int64_t ssd_read_bytes, ssd_write_bytes;
  int64_t host_hits, host_misses;         /* host cache lookups for S+ and sync fetches */
  int64_t sync_fetches;                   /* blocks of K_t that were not on the GPU in time */
  double stall_seconds;                   /* host time blocked in tide_ensure_resident */
  int64_t resident;                       /* |R_t| */
  int64_t prefetch_issued, prefetch_used; /* hinted blocks read ahead / later admitted */
  int64_t skipped;                        /* blocks of K_t left out of the render (BOUNDED) */
} tide_tier_stats;

/* Creates the tier over pool (n_slots >= cfg->capacity; block_rows = B).
 * No file is touched: a new store is laid out with tide_store_put_block /
 * tide_store_finalize, an existing one is loaded with tide_store_open.
 * d_spheres: f32 [K][4] (cx, cy, cz, r) and d_dirty: u8 [K], K = ceil(N/B),
 * both device memory (host memory with TIDE_TIER_HOST_POOL); the tier keeps
 * host copies.  Nothing is resident after creation. */
tide_status tide_residency_create(const tide_store_cfg* cfg, tide_pool* pool, float* d_spheres,
                                  uint8_t* d_dirty, tide_residency** out);
tide_status tide_residency_destroy(tide_residency* res);

/* Layout order (Sec. 3.3): perm [n] = the rows sorted by the Morton code of
 * their centres (xyz at xyz + i * stride, host f32), stably (ties keep row
 * order).  Each axis is quantised to 2^21 cells over the centres' bounding
 * box; code bit 3i+a is bit i of axis a's cell index (a = 0, 1, 2 = x, y, z).
 * Block k of the layout is then rows perm[kB .. (k+1)B). */
tide_status tide_morton_order(const float* xyz, int64_t n, int64_t stride, int64_t* perm);

/* Out-of-core layout build (Sec. 3.3, 4.1) of a new store: table_path holds
 * the N rows of the tier as f32 [N][59], row-major (N and B from the tier's
 * configuration).  Pass 1 reads the centres' bounding box; pass 2 sorts runs
 * of run_rows rows by (Morton code, row), with tide_morton_order's
 * quantisation, into files under tmp_dir; pass 3 merges the runs and writes
 * every block through tide_store_put_block, then tide_store_finalize.  The
 * block contents equal those of tide_morton_order's permutation.  Host
 * memory is about 490 B per run row; at most 512 runs; the run files are
 * removed on return.  TIDE_EINVAL if the file size is not N * 236 B or a
 * centre is not finite; TIDE_EIO on a read or write error. */
tide_status tide_layout_build(tide_residency* res, const char* table_path, const char* tmp_dir, int64_t run_rows);

/* Training-view order (Sec. 3.5 and App. A: a clustered travelling-salesperson
 * order of the camera poses, so that consecutive batches share blocks).
 * perm [n] receives a permutation of the n cameras:
 *   d(i, j) = |p_i - p_j| + dir_weight |f_i - f_j| (p = -R^T t the centre,
 *   f = R's third row the viewing direction, dir_weight in metres);
 *   ceil(n / cluster_size) clusters of the centres (farthest-point seeds
 *   from camera 0, Lloyd iterations until stable, at most 100);
 *   the non-empty clusters along an open path over their centroids from
 *   camera 0's cluster (nearest neighbour, then 2-opt);
 *   inside each, an open path with d entered at the camera nearest the
 *   previous cluster's last (camera 0 first), nearest neighbour then 2-opt.
 * Ties go to the lower index; a 2-opt move must gain more than 1e-9.
 * Deterministic; host only. */
tide_status tide_view_order(const tide_camera* cams, int64_t n, int32_t cluster_size, double dir_weight,
                            int32_t* perm);

/* Layout build (Sec. 3.3, 4.1): writes block k's record to the base segment
 * with zero moments and steps (only the parameters are written; the new
 * segment's moments and steps are holes that read as zeros).  params: host
 * f32 [59][rows of block k].
 * Computes the block's sphere: c_k = mean of the member means (fixed),
 * r_k = max |mu_i - c_k| + 3 kappa max exp(log-scale_i). */
tide_status tide_store_put_block(tide_residency* res, int64_t block, const float* params);
/* Ends the layout build: persists Index and uploads the spheres. */
tide_status tide_store_finalize(tide_residency* res);
/* Reopens an existing store (after tide_residency_create on the same dir):
 * loads the persisted Index and the sphere file. */
tide_status tide_store_open(tide_residency* res);

/* Level 1: K^(c) for each camera.  out_ids receives the ascending block ids
 * of camera 0, then camera 1, ...; counts[c] their numbers.  cap = capacity
 * of out_ids; TIDE_ECAPACITY if it is too small. Uses the host spheres. */
tide_status tide_cull_blocks(const tide_residency* res, const tide_camera* cams, int32_t n_cams,
                             int32_t* out_ids, int32_t* counts, int64_t cap);

/* Makes every block of K (ascending ids) resident and writes the pool's
 * order array (slots of K in ascending block id) and n_order; the compute
 * stream waits for the transfers.  Host-blocking time is added to
 * stall_seconds (and returned in *stall_s if non-null).  With
 * TIDE_TIER_BOUNDED the order array holds the resident blocks of K only. */
tide_status tide_ensure_resident(tide_residency* res, const int32_t* K, int32_t n, void* compute_stream,
                                 double* stall_s);

/* Alg. 1 with the per-camera next sets; enqueues S- device-to-host copies
 * behind the compute event of the current iteration, and S+ host-to-device
 * copies (SSD reads on the I/O threads first).  out_plus / out_minus
 * (capacity cap each, may be null) receive S+ and S-. */
tide_status tide_stream_delta(tide_residency* res, const int32_t* knext_ids, const int32_t* knext_counts,
                              int32_t n_cams, void* side_stream, int32_t* out_plus, int32_t* n_plus,
                              int32_t* out_minus, int32_t* n_minus, int64_t cap);

/* Records the end of iteration t's compute on compute_stream and enqueues
 * the read-back of spheres and dirty flags. */
tide_status tide_residency_end_iteration(tide_residency* res, void* compute_stream);
/* Waits for that read-back; the next culling uses the refreshed bounds. */
tide_status tide_residency_sync_bounds(tide_residency* res);

/* Prefetch hint: read these blocks (most urgent first) from the SSD into the
 * host cache ahead of need, as speculative reads that the I/O threads serve
 * only when no demand read or write-back is waiting.  Resident and cached
 * blocks are skipped.  At most 2 x io_threads speculative reads are
 * outstanding and a hint only takes a clean, idle host entry that was not
 * filled by a prefetch in the last 4 iterations; the rest of the list is
 * dropped (hints are meant to be renewed every iteration).  horizon =
 * iterations ahead, informational. */
tide_status tide_prefetch_hint(tide_residency* res, const int32_t* blocks, int32_t n, int32_t horizon);

/* Consistency barrier (Sec. 3.4): device-to-host of every dirty resident
 * block, flush of every dirty host entry to a patch segment, fsync, then the
 * Index is persisted atomically. Blocks until done. */
tide_status tide_checkpoint(tide_residency* res);

/* Compaction (Sec. 3.4, off the training path): a checkpoint, then the
 * newest version of every block is rewritten in block order into a new base
 * segment that replaces the old by rename; the Index is persisted pointing
 * there (versions kept) and the patch segments are deleted.  Crash-safe at
 * every step (the old Index stays valid until the new one is in place).
 * Called between iterations (after tide_residency_sync_bounds); blocks until
 * done. */
tide_status tide_store_compact(tide_residency* res);

/* Reads block k's newest record (host, rec_bytes) through Index: from the
 * GPU if resident (blocking copy), else the host cache, else the SSD. */
size_t tide_block_record_bytes(int32_t block_rows);
tide_status tide_read_block(tide_residency* res, int64_t block, void* dst);

tide_status tide_tier_get_stats(const tide_residency* res, tide_tier_stats* out);
/* Host copy of the spheres (f32 [K][4]) as the tier currently sees them. */
tide_status tide_tier_spheres(const tide_residency* res, float* out, int64_t n_blocks);
/* The resident set R (Sec. 3.5) as the tier's host tables hold it: ascending
 * block ids into out (capacity cap), their number in *n; TIDE_ECAPACITY if
 * cap is too small.  Host-only (no device synchronisation). */
tide_status tide_tier_resident(const tide_residency* res, int32_t* out, int64_t cap, int32_t* n);

/* ------------------------------------------------------------------------
 * Learned prefetch predictor.  Not part of the paper's method: a small ReLU
 * MLP maps the recent camera poses to per-block visibility for the next few
 * iterations, so that the SSD reads of blocks about to enter the working set
 * start early (host prefetch via tide_prefetch_hint).  Exact Level-1 culling
 * (Sec. 3.3, Eq. for K_t) stays in charge of what is rendered: a block the
 * predictor misses is streamed by Alg. 1 as before, so rendered results do
 * not depend on it.
 *
 * Network: n_layers affine layers of widths dims[0] -> dims[1] -> ... ->
 * dims[n_layers]; ReLU after every layer but the last, whose outputs are
 * logits (sigmoid = visibility probability).  Every width is a positive
 * multiple of 8; dims[n_layers] is a multiple of 32 (label bitsets).
 *
 * Parameter layout (one flat buffer, P = tide_mlp_param_count()): for each
 * layer l in order, W_l f32 [dims[l+1]][dims[l]] row-major, then b_l f32
 * [dims[l+1]].  params is the FP32 master copy; params_bf16 holds the same
 * values rounded to bfloat16 (nearest, ties to even; uint16 bit patterns);
 * the products read W from params_bf16 and the biases from params.
 * Activations, gradients and accumulation are FP32.  The products run on
 * the bf16 matrix cores: an FP32 operand is split into a bf16 pair
 * (hi = bf16(a), lo = bf16(a - hi)) and both halves are multiplied, so each
 * product keeps about 16 significant bits of the FP32 operand.
 * ---------------------------------------------------------------------- */
#define TIDE_MLP_MAX_LAYERS 8

typedef struct {
  int32_t n_layers;
  int32_t dims[TIDE_MLP_MAX_LAYERS + 1];
  float* params;          /* device f32 [P], FP32 master (16-byte aligned) */
  uint16_t* params_bf16;  /* device bf16 bits [P] (16-byte aligned) */
  float* grad;            /* device f32 [P], written by tide_mlp_bwd */
  float* exp_avg;         /* device f32 [P], Adam first moment */
  float* exp_avg_sq;      /* device f32 [P], Adam second moment */
  int64_t step;           /* Adam steps taken; tide_mlp_adam increments it */
} tide_mlp;

/* Number of parameters P, or -1 if dims are invalid. */
int64_t tide_mlp_param_count(const int32_t* dims, int32_t n_layers);
/* Workspace of tide_mlp_fwd / tide_mlp_bwd for a batch: the hidden
 * activations of the forward (kept for the backward), the backward's
 * gradient buffers and the loss partial sums. */
size_t tide_mlp_ws_bytes(const tide_mlp* mlp, int32_t batch);
/* params_bf16 <- bf16(params) (after initialising or loading params). */
tide_status tide_mlp_sync_bf16(const tide_mlp* mlp, void* stream);
/* logits f32 [batch][dims[L]] = MLP(x), x f32 [batch][dims[0]], both device
 * and row-major.  Keeps the hidden activations in ws for tide_mlp_bwd. */
tide_status tide_mlp_fwd(const tide_mlp* mlp, const float* x, int32_t batch, float* logits, void* ws,
                         size_t ws_bytes, void* stream);
/* Binary cross-entropy with logits, averaged over batch x (valid outputs):
 *   l(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)).
 * label_bits u32 [batch][dims[L] / 32] (bit o % 32 of word o / 32 = label of
 * output o), valid_bits u32 [dims[L] / 32] (outputs that count; padding
 * blocks are 0), both device.  Must follow tide_mlp_fwd with the same x,
 * batch and ws; logits is its output.  Writes the mean loss to d_loss
 * (device f64 scalar) and overwrites mlp->grad with its gradient. */
tide_status tide_mlp_bwd(const tide_mlp* mlp, const float* x, const float* logits, const uint32_t* label_bits,
                         const uint32_t* valid_bits, int32_t batch, double* d_loss, void* ws, size_t ws_bytes,
                         void* stream);
/* One Adam step on every parameter from mlp->grad (no weight decay):
 *   m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
 *   p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),   t = ++step;
 * then params_bf16 <- bf16(params). */
tide_status tide_mlp_adam(tide_mlp* mlp, float lr, float beta1, float beta2, float eps, void* stream);
/* Threshold: out_bits u32 [batch][n_out / 32], bit set where
 * logits >= threshold_logit (the logit of the probability threshold). */
tide_status tide_mlp_predict_bits(const float* logits, int32_t batch, int32_t n_out, float threshold_logit,
                                  uint32_t* out_bits, void* stream);

/* Host helpers of the predictor's data path.
 * tide_pose_features: one feature row per history of n_poses consecutive
 * cameras (oldest first): per pose the 12 values of [R | t / t_scale]
 * (R row-major, then t), then the ground-plane (x, y) displacement of the
 * camera centre from the previous pose (0 for the first), 14 floats per
 * pose; out f32 [n_poses * 14].
 * tide_cull_bits: union over n_cams cameras of the Level-1 block sets for
 * the given spheres (f32 [K][4], same six-plane test as tide_cull_blocks),
 * as a bitset out u32 [n_words] (bit k % 32 of word k / 32; words past K are
 * zero); n_words >= ceil(K / 32).
 * tide_block_sphere: the bounding sphere tide_store_put_block computes for a
 * block (Sec. 3.3): params holds the block's first six parameter columns
 * (mean xyz, log-scale xyz), column j at params + j * ld, rows <= ld;
 * out f32 [4] = (cx, cy, cz, r). */
tide_status tide_pose_features(const tide_camera* cams, int32_t n_poses, double t_scale, float* out);
tide_status tide_cull_bits(const float* spheres, int64_t n_blocks, const tide_camera* cams, int32_t n_cams,
                           uint32_t* out, int64_t n_words);
tide_status tide_block_sphere(const float* params, int64_t ld, int64_t rows, double kappa, float* out);

/* ------------------------------------------------------------------------
 * Timing hook for measurement.  Arms a pair of caller-created HIP events
 * (hipEvent_t) for one kernel of the library; every later launch of that
 * kernel records ev_start immediately before and ev_stop immediately after
 * it, on the launch stream, until tide_timer_clear().  Kernel names:
 * "preprocess", "compact_vis", "radix_scatter", "emit", "render_fwd",
 * "loss_fwd", "loss_bwd", "render_bwd", "reduce_pairs", "adjoint", "adam",
 * "adjoint_adam".
 * At most 16 names are armed at once; re-arming a name replaces its events.
 * The events are not owned by the library.
 * ---------------------------------------------------------------------- */
tide_status tide_timer_arm(const char* kernel, void* ev_start, void* ev_stop);
tide_status tide_timer_clear(void);

#ifdef __cplusplus
}
#endif
#endif /* TIDE_H */
