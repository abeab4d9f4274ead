// Device-side descriptors of the consensus, quantizer and regularization
// kernels of the tomoadmm HIP library (gfx950).
#pragma once

#include "common.h"

namespace tomo {

// ---------------------------------------------------------------------------
// Consensus / quantization: one job = one segment of one node.
// ---------------------------------------------------------------------------
struct SegJob {
  float* x;             // slice consensus image [n][n]
  const float* u;       // this node's u (SEG mode)
  const float* lam;     // this node's lambda (SEG mode)
  const float* tz;      // regularization block's target z + nu / rho_z [n][n], or null
  float rho_z;          // its penalty
  int n, row0, rows;
  float rho, eta2;
  // AVG mode: the slice's nodes are nodes[node0 .. node0 + n_nodes)
  int node0, n_nodes;
  // message outputs (nullable)
  uint8_t* labels;
  float* centroids;
  int32_t* iters;
  int16_t* coeffs;
  float* lohi;
  float* xt;            // the segment before Q (nullable)
  // DCT codec (k_dct_range, then k_dct_code): the matrix coded is src[rows][cols]
  // with leading dimension ld, written to dst (in the consensus both are the
  // segment of x, ld = cols = n)
  const float* src;
  float* dst;
  int cols, ld;
  int chunk_rows, n_chunks;   // range partials: rows per chunk, chunks (<= DCT_MAX_CHUNKS)
  float4* part;               // [n_chunks] (lo, hi, non-finite flag, unused)
  int range_wg, code_wg;      // first workgroup of the job in the two launches
};

// DCT codec launch shapes: the range launch gives each workgroup at least
// DCT_CHUNK values (whole rows) and a segment at most DCT_MAX_CHUNKS
// workgroups; the coding launch gives each workgroup a strip of 16 rows x
// DCT_STRIP columns (a 16 x 64 sub-strip per wave).
constexpr int DCT_THREADS = 256;
constexpr int DCT_CHUNK = 4096;
constexpr int DCT_MAX_CHUNKS = 64;
constexpr int DCT_STRIP = 256;
__host__ __device__ inline int dct_chunk_rows(int rows, int cols) {
  const int a = (DCT_CHUNK + cols - 1) / cols, b = (rows + DCT_MAX_CHUNKS - 1) / DCT_MAX_CHUNKS;
  return a > b ? a : b;
}
__host__ __device__ inline int dct_code_wgs(int rows, int cols) {
  return ((rows + 15) / 16) * ((cols + DCT_STRIP - 1) / DCT_STRIP);
}

struct NodeRef {        // u, lambda of one node (AVG gather, dual update)
  float* u;
  float* lam;
  const float* x;
  int n;
  float rho;
  int wg_begin;
};

struct AvgJob {         // x = mean over nodes[node0 .. node0+n_nodes) of u + lambda/rho
  float* x;
  const float* tz;      // regularization block's target, or null (then the plain mean)
  float rho_z;
  int node0, n_nodes, n;
  int wg_begin;
};

// K-means over segments: one job per segment (see kmeans.hip)
constexpr int KM_MAX_K = 256;

struct KMJob {
  const float* src;     // values (the segment of x in the consensus step)
  float* x;             // where the x-updated values are stored (consensus)
  float* a_hat;         // quantized values (nullable, may equal src)
  const float* u;       // Alg. 3 inputs, or null for no x-update
  const float* lam;
  uint8_t* labels;      // [n] (nullable)
  float* cent;          // [k] (nullable)
  int32_t* iters;       // [1] (nullable)
  float* work;          // [n] regrouping workspace, required when n > KM_LDS_VALUES
  float* xt;            // [n] the values before Q (nullable)
  long long n;          // < 2^31
  float rho, eta2;
};

// A K-means job's regularization block: the target t_z of its segment (or
// null) and the block's penalty; a table parallel to the jobs, read only by the
// kernel instantiation for calls with blocks.
struct KMBlock {
  const float* tz;
  float rho_z;
};

// Segments up to this many values are regrouped in LDS; longer ones in the
// job's global workspace of n floats.
constexpr int KM_LDS_VALUES = 16384;

// ---------------------------------------------------------------------------
// Regularization block (one per slice): z = prox_{theta R}(x - nu / rho_z),
// theta = mu / rho_z; R Tikhonov (1/2 ||z||^2) or isotropic TV by Chambolle's
// dual projection iterations on the field (p1, p2), ping-ponged per launch
// between the caller's buffer (slot 0) and a library scratch buffer (slot 1).
// ---------------------------------------------------------------------------
enum { REG_TIKHONOV = 1, REG_TV = 2 };
constexpr int TV_BLOCK = 6;     // most Chambolle iterations per k_reg_step launch (and its halo width)
// k_reg_step: one workgroup per tile of 20 rows x (64 - 2 TV_BLOCK) columns
constexpr int TV_TILE_H = 20, TV_TILE_W = 64 - 2 * TV_BLOCK;
constexpr int TV_THREADS = 1024; // threads per k_reg_step workgroup: two region rows per thread

// Launches of one TV z-update of T Chambolle iterations: the fewest that run at
// most TV_BLOCK iterations each and at most TV_BLOCK - 1 in the last, rounded up
// to an even count (so that the field ends in the slot it started from); one
// launch when T = 0 (z from the field as it is).
__host__ __device__ inline int tv_launches(int T) {
  return T == 0 ? 1 : ((T / TV_BLOCK + 2) & ~1);
}
// iterations of launch l of L: T spread evenly, the remainder on the first ones
__host__ __device__ inline int tv_launch_iters(int T, int L, int l) {
  return T / L + (l < T % L ? 1 : 0);
}

// Alg. 3 on one value: E2 gradient steps x <- x - eta2 rho (x - t_m), t_m = u +
// lambda/rho formed once per value (reg_target); with a block's term
// x <- x - eta2 (rho (x - t_m) + rho_z (x - t_z)).  The objective is quadratic in
// x, so the steps are a linear recurrence with factor a = 1 - eta2 s, s = rho
// (+ rho_z), and E2 of them equal x + (1 - a^E2) (t - x) for the fixed point t
// = (rho t_m + rho_z t_z) / s.  The kernels apply that closed form: without a
// block x + q (t_m - x) with q = 1 - a^E2, with one x + c (rho (t_m - x) + rho_z
// (t_z - x)) with c = q / s; the coefficients are formed once in float64 and
// rounded to float32, and every kernel running the update rounds the same way.
// E2 = 0 leaves x as it is (callers skip the update).
__device__ __forceinline__ float reg_target(float uv, float lv, float irho) { return fmaf(lv, irho, uv); }
__device__ __forceinline__ double xseg_decay(double s, float eta2, int e2) {   // a^E2
  const double a = 1.0 - (double)eta2 * s;
  double p = 1.0;
  for (int e = 0; e < e2; ++e) p *= a;
  return p;
}
__device__ __forceinline__ float xseg_q(float rho, float eta2, int e2) {
  return (float)(1.0 - xseg_decay((double)rho, eta2, e2));
}
__device__ __forceinline__ float xseg_c(float rho, float rho_z, float eta2, int e2) {
  const double s = (double)rho + (double)rho_z;
  return (float)((1.0 - xseg_decay(s, eta2, e2)) / s);
}
__device__ __forceinline__ float xseg(float xv, float tm, float q) { return fmaf(q, tm - xv, xv); }
__device__ __forceinline__ float xseg_reg(float xv, float tm, float tv, float rho, float rho_z, float c) {
  return fmaf(c, fmaf(rho, tm - xv, rho_z * (tv - xv)), xv);
}

struct RegJob {
  const float* x;       // slice consensus image [n][n]
  const float* nu;      // block dual
  float* z;             // block copy (output)
  float* tz;            // v = x - nu / rho_z during the iterations, then z + nu / rho_z
  float* p[2];          // TV dual field slots, each [2][n][n] (p1 then p2)
  int n, kind, iters;
  float theta, irho_z, tau;
  int wg_begin;
};

}  // namespace tomo
