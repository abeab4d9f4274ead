/*
 * tomoadmm.h -- C ABI of the MI355X (gfx950) library for decentralized ADMM
 * tomographic reconstruction with quantized exchange.
 *
 * Method: "Distributed Tomographic Reconstruction with Quantization"
 * (arXiv 2410.06106).  The library computes, on one GPU, the per-node work of
 * the paper's decentralized ADMM: the local u-update (Alg. 2), the segment
 * x-update (Alg. 3) or the averaging x-update (Eq. 9), the quantizer Q of the
 * exchanged segments (Alg. 5 and the JPEG-style codec), the concatenation
 * (Eq. 23) and the dual update (Eq. 24).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller (for example
 *   the storage of a torch tensor).  The library never frees caller memory.
 * - Images are float32 [n][n], row-major.  Pixel (r, c) has its centre at
 *   x = c - (n-1)/2, y = r - (n-1)/2 in pixel units; y grows with the row index.
 * - Sinograms are float32 [n_ang][n_bins], row-major; bin b is centred at
 *   t = b - (n_bins-1)/2.  Angles are float64 radians; the ray (theta, t) is the
 *   line x cos(theta) + y sin(theta) = t (Section 2.1, Eq. 1).
 * - System matrix (Eq. 2-4, Joseph linear-interpolation discretisation):
 *     P[(theta,b),(r,c)] = max(0, 1 - |t_b - t_rc| / c_theta) / c_theta,
 *     t_rc = x_c cos(theta) + y_r sin(theta), c_theta = max(|cos|, |sin|).
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *   only enqueues work on that stream and returns; nothing blocks the host
 *   except the first use of a new node list (see admm_local_update).
 * - Return value: TOMO_OK, or an error code.  Argument errors (TOMO_EINVAL) are
 *   detected on the host before anything is enqueued.  A failed kernel launch
 *   returns TOMO_EDEVICE.  tomo_last_error() describes the latest failure of a
 *   context in words.  No C++ exception crosses this interface.
 * - A context owns reusable device workspace.  Calls made with one context must
 *   be issued from one host thread and ordered on one stream at a time.
 */
#ifndef TOMOADMM_H
#define TOMOADMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tomo_ctx tomo_ctx;

enum {
  TOMO_OK = 0,
  TOMO_EINVAL = 1,        /* bad argument, checked on the host                 */
  TOMO_ENOMEM = 2,        /* device workspace could not be allocated            */
  TOMO_EDEVICE = 3,       /* HIP runtime or kernel launch failure               */
  TOMO_EUNSUPPORTED = 4   /* valid request the library does not handle         */
};

/* Create a context bound to HIP device `device`.  *ctx receives the handle. */
int tomo_create(tomo_ctx** ctx, int device);
/* Release the context and its workspace (waits for its pending work). */
int tomo_destroy(tomo_ctx* ctx);
/* Static text for a status code. */
const char* tomo_status_string(int status);
/* Text of the latest error recorded on `ctx` ("" if none). */
const char* tomo_last_error(const tomo_ctx* ctx);
/*
 * Free the context's cached plans (one per node list seen by
 * admm_local_update / admm_consensus, kept so later calls and captured graphs
 * reuse them) and its standalone workspaces.  Waits for the device first.
 * Graphs captured before this call must not be replayed afterwards; the next
 * call of each kind allocates again.  Workspaces otherwise only grow: an
 * allocation a larger request replaces is kept until tomo_release or
 * tomo_destroy, so earlier captured graphs stay valid.
 */
int tomo_release(tomo_ctx* ctx);

/*
 * Launch-shape options of a context (the tile choices an autotuner varies).
 * Values take effect for plans built afterwards: setting an option retires the
 * context's cached plans (their memory stays allocated until tomo_destroy, so
 * graphs captured earlier remain valid).  Results do not depend on the options except for
 * floating-point summation order in the projector (regions are added in a
 * fixed order, so a given option value is bit-reproducible).
 *   TOMO_OPT_PROJ_JOB_WGS   projector workgroups wanted per node before its
 *                           image is split into smaller regions (default 16,
 *                           1 .. 65536)
 *   TOMO_OPT_PROJ_BAND      image lines the projector stages in LDS per pass
 *                           (16 or 32, default 32); changes the projector's
 *                           summation order only
 *   TOMO_OPT_PROJ_KERNEL    0: band-streamed projector (the two options above
 *                           apply); 1: region-resident projector (one
 *                           workgroup per 128 x 128 region holds it in LDS for
 *                           every angle of the node; images up to 2048 x 2048,
 *                           larger ones use kernel 0).  Default 0.
 *   TOMO_OPT_PROJ_MODEL     system matrix of every projector and backprojector
 *                           call of the context: 0 (default) the Joseph weights
 *                           stated above; 1 the intersection lengths Eq. 2 names:
 *                           P[(theta,b),(r,c)] = length of the line of bin b
 *                           inside the unit square of pixel (r, c), which with
 *                           D = t_b - t_rc is the trapezoid
 *                           h * clamp((w2 - |D|) / (w2 - w1), 0, 1),
 *                           h = 1 / max(|cos|,|sin|), w1 = ||cos| - |sin|| / 2,
 *                           w2 = (|cos| + |sin|) / 2.  A cos or sin within 1e-12
 *                           of zero counts as zero; a line along a pixel edge
 *                           then belongs to the pixel on its +x (+y) side
 *                           (half-open pixels).  Model 1 always uses the
 *                           band-streamed projector and computes positions in
 *                           float64 (about twice the cost).
 *   TOMO_OPT_PROJ_ORDER     dispatch order of the band-streamed projector
 *                           of admm_local_update / admm_local_phase: with 1,
 *                           a launch of at most 8 workgroups per compute
 *                           unit starts its workgroups in an order the plan
 *                           derives from a cost it estimates from the node
 *                           angles (read back to the host once, when the
 *                           plan is built): per die, largest first; with 2
 *                           (default), the same with all workgroups of a node
 *                           on one die, and, when every die then receives the
 *                           same number of them, the node's region-reduction
 *                           and backprojector workgroups on that die too (each
 *                           die then reads the data of its own nodes only);
 *                           larger launches, and 0, keep node order.  Results
 *                           are bit-identical for all values.
 */
enum {
  TOMO_OPT_PROJ_JOB_WGS = 1,
  TOMO_OPT_PROJ_BAND = 3,
  TOMO_OPT_PROJ_KERNEL = 4,
  TOMO_OPT_PROJ_MODEL = 5,
  TOMO_OPT_PROJ_ORDER = 6
};
int tomo_set_option(tomo_ctx* ctx, int32_t option, int64_t value);

typedef struct {
  int32_t n;       /* image side: the image is n x n pixels (1 <= n <= 4096) */
  int32_t n_bins;  /* detector bins per angle (n_bins >= 1)                  */
} tomo_geom;

/*
 * Forward projection d = P u (Eq. 2-4) over `n_ang` angles.
 *   angles: float64 [n_ang];  image: float32 [n][n];  sino: float32 [n_ang][n_bins]
 * sino is overwritten.  image and sino must not overlap.  n_ang == 0 is a no-op.
 */
int tomo_project(tomo_ctx* ctx, tomo_geom g, const double* angles, int32_t n_ang,
                 const float* image, float* sino, void* stream);

/*
 * Matched backprojection, the exact transpose of tomo_project:
 *   image = alpha * P^T sino + beta * image
 * (image is not read when beta == 0).  Same layouts as tomo_project.  With
 * n_ang == 0 the sinogram is empty and P^T sino is zero: image = beta * image
 * (zeros when beta == 0); angles and sino may then be null.
 */
int tomo_backproject(tomo_ctx* ctx, tomo_geom g, const double* angles, int32_t n_ang,
                     const float* sino, float* image, float alpha, float beta, void* stream);

/*
 * Batches of independent projections / backprojections, one launch per kernel
 * for the whole batch (for example the per-node operators of an unrolled,
 * differentiated ADMM).  Each item has its own geometry, angles, image and
 * sinogram:
 *   tomo_project_many:      items[i].sino  = P_i items[i].image
 *   tomo_backproject_many:  items[i].image = alpha P_i^T items[i].sino + beta items[i].image
 * with the layouts of tomo_project.  Results are bit-identical to one
 * tomo_project / tomo_backproject call per item.  Nothing is cached: every call
 * builds the batch's job table on the host and copies it to the device on
 * `stream` through pinned staging memory of the context (the item pointers
 * may change from call to call, as they do in an autograd graph); because of
 * that copy, do not capture these two calls into a HIP graph.
 * Errors: TOMO_EINVAL for an empty list, an invalid item (geometry, n_ang < 1,
 * null pointer) or an output overlapping any item's input or another output.
 */
typedef struct {
  tomo_geom g;
  const double* angles;   /* float64 [n_ang]                                   */
  int32_t n_ang;          /* >= 1                                              */
  int32_t reserved;       /* must be 0 (keeps the struct free of padding)       */
  float* image;           /* float32 [n][n]                                    */
  float* sino;            /* float32 [n_ang][n_bins]                           */
} tomo_proj_item;

int tomo_project_many(tomo_ctx* ctx, const tomo_proj_item* items, int32_t n_items, void* stream);
int tomo_backproject_many(tomo_ctx* ctx, const tomo_proj_item* items, int32_t n_items, float alpha,
                          float beta, void* stream);

/*
 * Centralized tomographic reconstruction by gradient descent (Section 2.2,
 * Alg. 1, minimising 0.5 ||P u - d||^2 of Eq. 5):
 *   repeat `iters` times:  u <- u - eta * P^T (P u - d)
 * over all `n_ang` angles, starting from the u passed in (Alg. 1 starts from
 * zeros: pass a zeroed u).  Each step is one projection with the residual
 * fused into its epilogue and one matched backprojection that updates u in
 * place.
 *   angles: float64 [n_ang];  d: float32 [n_ang][n_bins];  u: float32 [n][n],
 *   read and overwritten.  u and d must not overlap.
 * Errors: TOMO_EINVAL for n_ang < 1, iters < 0, a non-finite eta, a null
 * pointer or overlapping u and d.  iters == 0 is a no-op.  The residual lives
 * in the context's workspace (n_ang * n_bins floats, allocated on the first
 * call that needs more).
 */
int tomo_ctr_gd(tomo_ctx* ctx, tomo_geom g, const double* angles, int32_t n_ang, const float* d,
                float* u, float eta, int32_t iters, void* stream);

/*
 * One node of the decentralized problem (Eq. 6-7): its angles and data d_m,
 * its local image u_m and dual variable lambda_m, the slice-wide consensus image
 * x, and the segment x[m] it owns (rows seg_row0 .. seg_row0+seg_rows-1 of x,
 * Eq. 13/17).  Nodes of one slice share `x` and must be adjacent in a node list;
 * the segments of one slice must not overlap, and the x arrays of different
 * slices must not overlap (TOMO_EINVAL otherwise: the consensus writes every
 * segment of every slice at the same time).
 */
typedef struct {
  tomo_geom g;
  const double* angles;   /* float64 [n_ang]                                   */
  int32_t n_ang;          /* >= 1                                              */
  int32_t slice;          /* slice id; equal ids <=> same x                     */
  const float* d;         /* float32 [n_ang][n_bins]  node data d_m             */
  float* u;               /* float32 [n][n]  u_m, updated in place              */
  float* lam;             /* float32 [n][n]  lambda_m, updated in place         */
  float* x;               /* float32 [n][n]  consensus image of the slice       */
  int32_t seg_row0;       /* first row of the owned segment                     */
  int32_t seg_rows;       /* rows in the owned segment (>= 1)                   */
  float rho;              /* penalty (> 0)                                      */
  float eta1;             /* step of Alg. 2                                     */
  float eta2;             /* step of Alg. 3                                     */
  int32_t reserved;       /* must be 0 (keeps the struct free of padding)       */
} tomo_node;

/*
 * Alg. 2 for every listed node: E1 steps of
 *   u_m <- u_m - eta1 * ( P_m^T (P_m u_m - d_m) + rho (u_m - x) + lambda_m )
 * starting from the current u_m (zero it before the first outer iteration).
 * n_nodes > 1 runs all nodes in one launch per step.  The first call with a
 * given node list (compared by value) builds a plan: it allocates workspace and
 * copies descriptors to the device synchronously, so capture a stream into a
 * graph only after one uncaptured call with the same list.
 */
int admm_local_update(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t e1,
                      void* stream);

/*
 * One launch of one half of an Alg. 2 step for every listed node (same plan as
 * admm_local_update), for timing and profiling the two kernels separately:
 *   phase 0: r_m = P_m u_m - d_m   into the plan's residual buffers;
 *   phase 1: u_m <- u_m - eta1 (P_m^T r_m + rho (u_m - x) + lambda_m).
 * admm_local_update with E1 = 1 is phase 0 followed by phase 1.
 */
int admm_local_phase(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t phase,
                     void* stream);

enum { TOMO_XUPDATE_SEGMENT = 0, TOMO_XUPDATE_AVERAGE = 1 };
enum { TOMO_QUANT_NONE = 0, TOMO_QUANT_KMEANS = 1, TOMO_QUANT_DCT = 2 };

typedef struct {
  int32_t kind;      /* TOMO_QUANT_*                                             */
  int32_t levels;    /* K-means clusters, 1..256                                 */
  int32_t max_iter;  /* K-means Lloyd iteration cap (>= 0)                       */
  int32_t quality;   /* DCT quality factor, 1..100                               */
} tomo_quant;

/* Optional per-node message buffers (device pointers, each may be NULL). */
typedef struct {
  uint8_t* labels;     /* K-means: uint8 [seg_rows*n] cluster index per value    */
  float* centroids;    /* K-means: float32 [levels]                              */
  int32_t* iters;      /* K-means: int32 [1] Lloyd iterations run                */
  int16_t* coeffs;     /* DCT: int16 [seg_rows][n] quantized coefficients        */
  float* lohi;         /* DCT: float32 [2] level-map range                       */
  float* x_tilde;      /* float32 [seg_rows][n]: the segment after the x-update  */
                       /* and before Q (Alg. 3 or Eq. 9 output; any quantizer)   */
} tomo_msg;

/*
 * Consensus, exchange and dual steps of one outer iteration, for every listed
 * node (all nodes of each listed slice must be present):
 *   mode TOMO_XUPDATE_SEGMENT: node m runs Alg. 3 on its own segment, E2 steps
 *     x[m] <- x[m] - eta2 * rho * (x[m] - u_m[m] - lambda_m[m]/rho), from x^k[m];
 *   mode TOMO_XUPDATE_AVERAGE: x = mean_m (u_m + lambda_m/rho) (Eq. 9, E2 unused);
 * then each segment is replaced by Q(segment) in place (Eq. 23), and finally
 *   lambda_m <- lambda_m + rho (u_m - x)   for every node (Eq. 24).
 * q == NULL means no quantization.  msg == NULL or an array of n_nodes entries.
 * K-means requires seg_rows*n < 2^31 values per segment; DCT requires seg_rows
 * and n to be multiples of 8.
 */
int admm_consensus(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t mode,
                   int32_t e2, const tomo_quant* q, const tomo_msg* msg, void* stream);

/*
 * Regularization as one more ADMM block (the separate sub-problem that the
 * paper's discussion, Section 4, proposes without a formulation).  A slice may
 * carry one block: a copy z of its image with its own dual nu, adding
 *   mu R(z) + nu^T (z - x) + rho_z/2 ||z - x||^2
 * to the augmented Lagrangian (Eq. 7).  Per outer iteration:
 *   admm_reg_update      z = prox_{theta R}(x - nu/rho_z), theta = mu/rho_z, and
 *                        t_z = z + nu/rho_z (reads x and nu, i.e. x^k, nu^k);
 *   admm_consensus_reg   the x-update with the block's term (SEG: every Alg. 3
 *                        step of a segment becomes
 *                        x <- x - eta2 (rho (x - u - lambda/rho) + rho_z (x - t_z));
 *                        AVG: x = (sum_m rho_m (u_m + lambda_m/rho_m) + rho_z t_z)
 *                        / (sum_m rho_m + rho_z)), the quantizer, Eq. 24 for every
 *                        node and nu <- nu + rho_z (z - x) for every block.
 * R: TOMO_REG_TIKHONOV, R(z) = 1/2 ||z||^2, prox v / (1 + theta); TOMO_REG_TV,
 * isotropic total variation sum_ij |(grad z)_ij| with forward differences that
 * vanish across the last row and column, its prox by tv_iters iterations of
 * Chambolle's dual projection algorithm (J. Math. Imaging Vis. 20, 2004):
 *   w = div p - v/theta,  p <- (p + tau grad w) / (1 + tau |grad w|),
 *   z = v - theta div p,
 * from the field p the block holds (warm start; zero it before the first
 * iteration), 0 < tau <= 0.25 (the convergence proof asks tau <= 1/8).
 * All pointers are device pointers the caller owns; z, nu, tz are float32
 * [n][n] and p float32 [2][n][n] (p1 then p2; TV only, else may be NULL), n
 * the slice's image side; they must not overlap each other or x.  The library
 * keeps one scratch field of 2 n^2 floats per TV block in a plan cached by the
 * block array (like the node plans; freed by tomo_release / tomo_destroy).
 * Errors: TOMO_EINVAL for a slice id no listed node has, two blocks of one
 * slice, an unknown kind, rho_z <= 0, mu < 0, tau outside (0, 0.25],
 * tv_iters outside [0, 10000] or a NULL pointer the kind needs.
 */
enum { TOMO_REG_TIKHONOV = 1, TOMO_REG_TV = 2 };

typedef struct {
  int32_t slice;     /* slice id (tomo_node.slice) the block belongs to        */
  int32_t kind;      /* TOMO_REG_TIKHONOV or TOMO_REG_TV                       */
  int32_t tv_iters;  /* Chambolle iterations per z-update (TV)                 */
  float mu;          /* weight of R (>= 0)                                     */
  float rho;         /* penalty rho_z of the constraint z = x (> 0)            */
  float tau;         /* Chambolle step (TV), 0 < tau <= 0.25                   */
  float* z;          /* float32 [n][n] the block's copy (written)              */
  float* nu;         /* float32 [n][n] its dual (updated by the consensus)     */
  float* tz;         /* float32 [n][n] z + nu/rho_z (written by the z-update)  */
  float* p;          /* float32 [2][n][n] TV dual field (read and written)     */
} tomo_reg;

int admm_reg_update(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, const tomo_reg* regs,
                    int32_t n_regs, void* stream);
int admm_consensus_reg(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t mode, int32_t e2,
                       const tomo_quant* q, const tomo_msg* msg, const tomo_reg* regs, int32_t n_regs,
                       void* stream);

/*
 * Scalar K-means quantizer (Alg. 5, Section 2.7) of a float32 vector a[n], bit-exact:
 *  lo,hi = min,max (NaN/Inf -> TOMO_EINVAL is NOT detectable on the host: the
 *  kernel then writes iters = -1 and leaves the outputs unspecified);
 *  centres start at lo + (hi-lo)(2j+1)/(2k) (float64, no FMA, rounded to float32);
 *  values enter the centroid sums as fixed point round(a * 2^S), S = 30 - e,
 *  e the binary exponent of max(|lo|,|hi|), summed exactly in int64;
 *  label = #{j < k-1 : 2a > c_j + c_{j+1}} in float64 (the nearest centre, the
 *  centres being kept in increasing order: after each update they are stably
 *  sorted; an empty cluster keeps its centre); Lloyd iterations until the
 *  labels repeat or max_iter.  hi == lo: labels 0, centres lo, iters 0.
 * Outputs: labels uint8 [n], centroids float32 [k] (increasing), a_hat float32
 * [n] (nullable, may alias a), iters int32 [1] (nullable).  1 <= k <= 256,
 * 1 <= n < 2^31.  Segments above 16384 values use a context workspace of
 * 4n bytes (allocated on first need, kept until tomo_destroy).
 */
int quantize_kmeans(tomo_ctx* ctx, const float* a, int64_t n, int32_t k, int32_t max_iter,
                    uint8_t* labels, float* centroids, float* a_hat, int32_t* iters, void* stream);

/*
 * Wire format of a K-means message (Section 2.6, Eq. 20; Section 3.3 counts a
 * K-level code as ceil(log2 K) bits).  tomo_pack_labels writes the n labels as
 * `bits`-bit codes: value i occupies bits [i*bits, (i+1)*bits) of a stream of
 * 32-bit words, least significant bit first, stream bit j being bit j mod 32 of
 * word j / 32; only the low `bits` bits of a label are stored and the last
 * word is padded with zeros.  A segment's message is this stream plus its
 * float32 codebook: 4 * ceil(n * bits / 32) + 4 * k bytes.
 *   labels: uint8 [n];  packed: uint32 [ceil(n*bits/32)], overwritten.
 * tomo_unpack_labels reads the stream back: labels[i] (nullable) and
 * a_hat[i] = centroids[code_i] (nullable; a code >= k reads centroids[k-1]).
 * Errors: TOMO_EINVAL for bits outside [1, 8], n outside [0, 2^31), a null
 * required pointer, a_hat without centroids or with k outside [1, 256], or an
 * output overlapping the input.  n == 0 is a no-op.
 */
int tomo_pack_labels(tomo_ctx* ctx, const uint8_t* labels, int64_t n, int32_t bits, uint32_t* packed,
                     void* stream);
int tomo_unpack_labels(tomo_ctx* ctx, const uint32_t* packed, int64_t n, int32_t bits,
                       const float* centroids, int32_t k, uint8_t* labels, float* a_hat, void* stream);

/*
 * Entropy code of DCT codes (the DCT message on the wire, Sections 2.6 and 2.7 / Eq. 20):
 * 8x8 blocks in row-major order; in a block the 64 int16 codes in zigzag order
 * (the scan order of baseline JPEG); the DC code sent as the difference from
 * the previous block's DC, differenced from 0 at the first block of every
 * restart interval of 64 blocks; the AC codes as pairs EG(zeros skipped + 1),
 * EG(2(|v| - 1) + (v < 0)) for every nonzero v, then EG(0) for the end of the
 * block; DC difference d as EG(2d) (d >= 0) or EG(-2d - 1) (d < 0).  EG(x) is
 * the order-0 Exp-Golomb code: floor(log2(x+1)) zero bits, then x + 1 in
 * binary.  Bits are packed most significant first: stream bit j is bit
 * 31 - (j mod 32) of words[j / 32]; unused bits are zero.
 *   coeffs: int16 [rows][ld] (row r, column c = coefficient (r mod 8, c mod 8)
 *   of block (r / 8, c / 8), as quantize_dct writes them); rows, cols
 *   multiples of 8.
 * tomo_dct_encode writes words (capacity max_words >= tomo_dct_encode_words,
 * all of it overwritten), restart: uint32 [ceil(blocks / 64)] bit offset of
 * each interval, and *total_bits (device uint32).  A message is the words in
 * use, the restart table and the level-map range: 4 ceil(total / 32) +
 * 4 ceil(blocks / 64) + 8 bytes.  Block offsets live in a context workspace
 * (4 bytes per block, allocated on first need).
 * tomo_dct_decode writes coeffs back from words[n_words], restart and
 * *total_bits (device), one thread per interval; a malformed stream ORs 1
 * into *status (device int32, nullable; it is not cleared).
 * Errors: TOMO_EINVAL for sizes that are not positive multiples of 8,
 * ld < cols, a null pointer, too small a words capacity or overlapping
 * arrays; TOMO_EUNSUPPORTED when blocks * 2302 >= 2^32.
 */
int64_t tomo_dct_encode_words(int32_t rows, int32_t cols);   /* ceil(blocks * 2302 / 32); 0 if invalid */
int tomo_dct_encode(tomo_ctx* ctx, const int16_t* coeffs, int32_t rows, int32_t cols, int32_t ld,
                    uint32_t* words, int64_t max_words, uint32_t* restart, uint32_t* total_bits,
                    void* stream);
int tomo_dct_decode(tomo_ctx* ctx, const uint32_t* words, int64_t n_words, const uint32_t* restart,
                    const uint32_t* total_bits, int32_t rows, int32_t cols, int32_t ld, int16_t* coeffs,
                    int32_t* status, void* stream);

/*
 * JPEG-style quantizer of a float32 matrix a[rows][cols] with leading dimension
 * ld (elements), the "standard JPEG" that Section 2.7 applies to an exchanged
 * segment as the Q of Eq. 23 (dADMM-J): per-matrix level map v = (a-lo)*255/(hi-lo) - 128, orthonormal
 * 8x8 DCT-II per block, codes = round-half-even(F / Qs) with Qs the ITU-T T.81
 * Table K.1 luminance table scaled to `quality` (scale 5000/q below 50, else
 * 200-2q; step = clamp(floor((T*scale+50)/100), 1, 255)), dequantize, inverse
 * DCT, unmap.  rows, cols multiples of 8.  Outputs: a_hat float32 [rows][ld]
 * (may alias a), coeffs int16 [rows][cols] (nullable), lohi float32 [2]
 * (nullable).  hi == lo: a_hat = a, coeffs 0.  A code within float32 error of
 * a rounding tie is decided on the coefficient recomputed in float64.  Two
 * launches over many workgroups (the range, then the coding); the range
 * partials live in a context workspace of 1 KiB (allocated on first use, kept
 * until tomo_destroy or tomo_release).
 */
int quantize_dct(tomo_ctx* ctx, const float* a, int32_t rows, int32_t cols, int32_t ld,
                 int32_t quality, int16_t* coeffs, float* a_hat, float* lohi, void* stream);

/*
 * quantize_dct for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and results, but the range partials live in a
 * library-owned device array of DCT_MAX_CHUNKS = 64 float4 (1 KiB) per GPU,
 * resolved by tomo_create and held until the process ends; no call allocates.
 * Every input size fits it (a matrix is cut into at most 64 row chunks); the
 * call still returns TOMO_EINVAL should a size need more.  All calls on one
 * GPU share that array and it keeps the last call's partials: calls that
 * overlap in time on one GPU (different streams, or contexts used from
 * different host threads) race and must be ordered by the caller.
 */
int quantize_dct_noalloc(tomo_ctx* ctx, const float* a, int32_t rows, int32_t cols, int32_t ld,
                         int32_t quality, int16_t* coeffs, float* a_hat, float* lohi, void* stream);

/*
 * Elementwise steps of the unrolled (differentiable) decentralized ADMM and
 * their exact gradients, for a learned penalty rho_k and step eta_k per
 * iteration.  The M nodes' images are stacked: U, L, B, G, dU, dL are float32
 * [M][npix], npix = n * n, node m at offset m * npix; x, dx are float32 [npix];
 * scal is float32 [2] in device memory = (rho, eta) (eta unused by the x-update
 * and dual calls); dscal is float32 [2] device output = (d rho, d eta).  All
 * pointers are device pointers owned by the caller; outputs must not overlap
 * inputs.  The scalar gradients are float64 sums reduced in a fixed order (a
 * context workspace of 96 KiB, allocated on first use).  Errors: TOMO_EINVAL
 * for m < 1, npix < 1, a null pointer or e2 < 0.
 *   tomo_unroll_ustep       Alg. 2 step: Uo = U - eta (B + rho (U - x) + L),
 *                           B = P^T (P U - D) computed by the caller with the
 *                           batched projector pair (tomo_axpby forms P U - D).
 *   tomo_unroll_ustep_grad  given G = dLoss/dUo, PG = P G, PtPG = P^T P G and the
 *                           forward residual R = P U - D (nsino values, stacked
 *                           like PG): dU = G - eta (PtPG + rho G), dL = -eta G,
 *                           dx = eta rho sum_m G_m, d rho = -eta <G, U - x>,
 *                           d eta = -(<PG, R> + rho <G, U - x> + <G, L>);
 *                           with accumulate != 0, dL, dx and dscal are added
 *                           to (the sums over several steps, in place).
 *   tomo_unroll_xseg        Alg. 3 on every row r from x: E2 steps
 *                           x <- x - eta2 rho (x - t), t = U_o + L_o / rho,
 *                           o = owner[r] (int32 [n], the node owning row r).
 *   tomo_unroll_xseg_grad   with a = 1 - eta2 rho: dx = a^E2 G, dU_o = (1 - a^E2) G,
 *                           dL_o = (1 - a^E2) G / rho (zero on rows a node does
 *                           not own), d rho = sum G ((1 - a^E2)(-L_o / rho^2)
 *                           - E2 eta2 a^(E2-1) (x - t)).
 *   tomo_unroll_seg_dual_grad  the two above chained, x' = xseg(U, L, x) and
 *                           L' = L + rho (U - x'), in one pass: given Gx =
 *                           dLoss/dx' (from its other uses) and GL = dLoss/dL',
 *                           with gx = Gx - rho sum_m GL_m: dL = GL + the xseg
 *                           term of gx, dU = rho GL + the xseg term of gx,
 *                           dx = a^E2 gx, d rho = sum_m <GL_m, U_m - x'> + the
 *                           xseg term; xs = x' (float32 [n][n]).
 *   tomo_unroll_xavg        Eq. 9: xo = (1/M) sum_m (U_m + L_m / rho).
 *   tomo_unroll_xavg_grad   dU_m = G / M, dL_m = G / (M rho),
 *                           d rho = -sum_m <G, L_m> / (M rho^2).
 *   tomo_unroll_dual        Eq. 24: Lo = L + rho (U - xn).
 *   tomo_unroll_dual_grad   dL = G, dU = rho G, dxn = -rho sum_m G_m,
 *                           d rho = <G, U - xn>.
 *   tomo_axpby              out = alpha a + beta b over n values (out may be a or b).
 *
 * The forward of one unrolled Alg. 2 step, fused into the batched projector
 * pair (two launches, the u-step in the backprojector's epilogue):
 *   tomo_unroll_local_step  items[i].sino = R_i = P_i U_i - D_i, then
 *                           Uo_i = U_i - eta (P_i^T R_i + rho (U_i - x) + L_i)
 *                           for the nodes of `items` (U_i = items[i].image, read
 *                           only; all items share n and n_bins).  D: float32
 *                           [sum n_ang][n_bins], the items' data rows in item
 *                           order; x float32 [n][n]; L, Uo float32
 *                           [n_items][n][n]; scal as above.  The job tables are
 *                           staged like tomo_project_many's (do not capture).
 *                           Errors: TOMO_EINVAL for an invalid item list,
 *                           items of different n or n_bins, a null pointer, or
 *                           an output (the R_i rows, Uo) overlapping an input
 *                           or the other output.
 */
int tomo_unroll_local_step(tomo_ctx* ctx, const tomo_proj_item* items, int32_t n_items, const float* D,
                           const float* x, const float* L, const float* scal, float* Uo, void* stream);
int tomo_axpby(tomo_ctx* ctx, int64_t n, float alpha, const float* a, float beta, const float* b, float* out,
               void* stream);
int tomo_unroll_ustep(tomo_ctx* ctx, int32_t m, int64_t npix, const float* U, const float* B, const float* x,
                      const float* L, const float* scal, float* Uo, void* stream);
int tomo_unroll_ustep_grad(tomo_ctx* ctx, int32_t m, int64_t npix, const float* G, const float* PtPG, const float* PG,
                           const float* R, int64_t nsino, const float* U, const float* x, const float* L,
                           const float* scal, float* dU, float* dL, float* dx, float* dscal, int32_t accumulate,
                           void* stream);
int tomo_unroll_xseg(tomo_ctx* ctx, int32_t m, int32_t n, const int32_t* owner, const float* U, const float* L,
                     const float* x, const float* scal, float eta2, int32_t e2, float* xo, void* stream);
int tomo_unroll_xseg_grad(tomo_ctx* ctx, int32_t m, int32_t n, const int32_t* owner, const float* G, const float* U,
                          const float* L, const float* x, const float* scal, float eta2, int32_t e2, float* dU,
                          float* dL, float* dx, float* dscal, void* stream);
int tomo_unroll_seg_dual_grad(tomo_ctx* ctx, int32_t m, int32_t n, const int32_t* owner, const float* Gx,
                              const float* GL, const float* U, const float* L, const float* x, const float* xs,
                              const float* scal, float eta2, int32_t e2, float* dU, float* dL, float* dx, float* dscal,
                              void* stream);
int tomo_unroll_xavg(tomo_ctx* ctx, int32_t m, int64_t npix, const float* U, const float* L, const float* scal,
                     float* xo, void* stream);
int tomo_unroll_xavg_grad(tomo_ctx* ctx, int32_t m, int64_t npix, const float* G, const float* L, const float* scal,
                          float* dU, float* dL, float* dscal, void* stream);
int tomo_unroll_dual(tomo_ctx* ctx, int32_t m, int64_t npix, const float* L, const float* U, const float* xn,
                     const float* scal, float* Lo, void* stream);
int tomo_unroll_dual_grad(tomo_ctx* ctx, int32_t m, int64_t npix, const float* G, const float* U, const float* xn,
                          const float* scal, float* dL, float* dU, float* dxn, float* dscal, void* stream);

/*
 * Sum of squared differences sum_i (a_i - b_i)^2 accumulated in float64 into
 * out[0] (overwritten).  Used for RMSE (Eq. 25) and relative-change traces.
 */
int tomo_sqdiff(tomo_ctx* ctx, const float* a, const float* b, int64_t n, double* out,
                void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TOMOADMM_H */
