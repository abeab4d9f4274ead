// Consensus, exchange and dual steps of decentralized ADMM (gfx950):
//   Alg. 3   segment x-update, E2 gradient steps on rho/2 ||u - x + lambda/rho||^2
//   Eq. 9    averaging x-update x = mean_m (u_m + lambda_m / rho)
//   JPEG-style quantizer: 8x8 DCT-II on MFMA, table quantization, inverse DCT
//   Eq. 24   dual update lambda_m += rho (u_m - x)
// One workgroup owns one segment for the x-update and the DCT quantizer, so a
// segment's level-map range never leaves the workgroup.  (The K-means quantizer
// lives in kmeans.hip.)
#include "consensus.h"

namespace tomo {

// ---------------------------------------------------------------------------
// workgroup reductions
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void wg_minmax(float& lo, float& hi, int& bad, float* red, int* redb) {
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { red[2 * w] = lo; red[2 * w + 1] = hi; redb[w] = bad; }
  __syncthreads();
  lo = red[0]; hi = red[1]; bad = redb[0];
  for (int i = 1; i < NT / 64; ++i) {
    lo = fminf(lo, red[2 * i]);
    hi = fmaxf(hi, red[2 * i + 1]);
    bad |= redb[i];
  }
}

// ---------------------------------------------------------------------------
// Alg. 3 on one segment (in place on x): E2 steps from the current x^k[m];
// with a regularization block its copy adds rho_z (x - t_z) to every step
// ---------------------------------------------------------------------------
// (xt: where the updated segment is copied as well, or null)
template <int NT>
__device__ void segment_xupdate(const SegJob& S, int e2, float* xt) {
  const size_t base = (size_t)S.row0 * S.n;
  const size_t cnt = (size_t)S.rows * S.n;
  const float irho = 1.f / S.rho;
  for (size_t i = threadIdx.x; i < cnt; i += NT) {
    float xv = S.x[base + i];
    const float tm = reg_target(S.u[base + i], S.lam[base + i], irho);
    if (S.tz) {
      const float tv = S.tz[base + i];
      for (int e = 0; e < e2; ++e) xv = xstep_reg(xv, tm, tv, S.rho, S.rho_z, S.eta2);
    } else {
      for (int e = 0; e < e2; ++e) xv = xstep(xv, tm, S.rho, S.eta2);
    }
    S.x[base + i] = xv;
    if (xt) xt[i] = xv;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// JPEG-style codec on MFMA, in two launches over many workgroups.
//
// k_dct_range: the segment's value range.  Each workgroup takes whole rows of
// one segment, runs the Alg. 3 x-update on them first (SEG mode; the updated
// values are stored back into x), and writes the chunk's (min, max,
// non-finite flag) to the job's partials.
//
// k_dct_code: each workgroup reduces its segment's partials (at most 64, one
// per lane, so every wave does it without a barrier) and codes a strip of 16
// rows.  A wave transforms one 16x16 tile = 2x2 blocks at a time with the
// block-diagonal matrix C2 = diag(C, C): with the tile X held in the
// accumulator layout of v_mfma_f32_16x16x4_f32 (lane j + 16 g, register r holds
// X[4g + r][j]) and passed as the A operand, one 4-instruction chain computes
// X^T B; two chains give C2 V C2^T forward and C2^T F C2 inverse.
//
// Rounding ties: a code is round-half-even(F / step) of the float64 DCT
// coefficient.  The float32 MFMA coefficient is within about 5e-4 of it (level
// map rounding plus two chained 8-term sums of values below 1024), so where
// F / step lies within 2e-3 / step of a half-integer the lane recomputes that
// coefficient in float64 from the block's values (the level map and the
// orthonormal DCT-II evaluated in float64) and rounds that instead.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

__constant__ unsigned char kLumaTable[64] = {
    16, 11, 10, 16, 24, 40, 51, 61,
    12, 12, 14, 19, 26, 58, 60, 55,
    14, 13, 16, 24, 40, 57, 69, 56,
    14, 17, 22, 29, 51, 87, 80, 62,
    18, 22, 37, 56, 68, 109, 103, 77,
    24, 35, 55, 64, 81, 104, 113, 92,
    49, 64, 78, 87, 103, 121, 120, 101,
    72, 92, 95, 98, 112, 100, 103, 99};

__device__ __forceinline__ double dct_coef64(int u, int x) {   // C[u][x], orthonormal DCT-II
  const double c = cos((double)((2 * x + 1) * u) * 3.14159265358979323846 / 16.0);
  return u == 0 ? sqrt(0.125) : c / 2.0;
}

__device__ __forceinline__ f4 mfma_chain(const f4& X, const float* B) {
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[0], B[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[1], B[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[2], B[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[3], B[3], acc, 0, 0, 0);
  return acc;
}

// the job owning workgroup bid of a launch, by the first-workgroup field F
// (jobs == null: the launch has the one job `single`)
template <int SegJob::*F>
__device__ __forceinline__ const SegJob* job_of(const SegJob* jobs, int n_jobs, const SegJob* single, int bid) {
  if (!jobs) return single;
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].*F <= bid) lo = mid; else hi = mid - 1;
  }
  return jobs + lo;
}

__global__ __launch_bounds__(DCT_THREADS) void k_dct_range(const SegJob* jobs, int n_jobs, SegJob single, int do_x,
                                                           int e2) {
  __shared__ float red[2 * (DCT_THREADS / 64)];
  __shared__ int redb[DCT_THREADS / 64];
  const SegJob& S = *job_of<&SegJob::range_wg>(jobs, n_jobs, &single, blockIdx.x);
  const int chunk = blockIdx.x - S.range_wg;
  const int r0 = chunk * S.chunk_rows, r1 = min(S.rows, r0 + S.chunk_rows);
  const int tid = threadIdx.x;
  const float irho = 1.f / S.rho;
  float lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int r = r0; r < r1; ++r) {
    for (int c = tid; c < S.cols; c += DCT_THREADS) {
      float v;
      if (do_x) {            // consensus: the segment of x, ld = cols = n
        const size_t i = (size_t)(S.row0 + r) * S.n + c;
        v = S.x[i];
        const float tm = reg_target(S.u[i], S.lam[i], irho);
        if (S.tz) {
          const float tv = S.tz[i];
          for (int e = 0; e < e2; ++e) v = xstep_reg(v, tm, tv, S.rho, S.rho_z, S.eta2);
        } else {
          for (int e = 0; e < e2; ++e) v = xstep(v, tm, S.rho, S.eta2);
        }
        S.x[i] = v;
      } else {
        v = S.src[(size_t)r * S.ld + c];
      }
      if (S.xt) S.xt[(size_t)r * S.cols + c] = v;
      bad |= !isfinite(v);
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
  }
  wg_minmax<DCT_THREADS>(lo, hi, bad, red, redb);
  if (tid == 0) S.part[chunk] = make_float4(lo, hi, bad ? 1.f : 0.f, 0.f);
}

__global__ __launch_bounds__(DCT_THREADS) void k_dct_code(const SegJob* jobs, int n_jobs, SegJob single,
                                                          int quality) {
  __shared__ double c64[64];
  const SegJob& S = *job_of<&SegJob::code_wg>(jobs, n_jobs, &single, blockIdx.x);
  const int lid = blockIdx.x - S.code_wg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < 64) c64[tid] = dct_coef64(tid >> 3, tid & 7);
  // the segment's range from its partials (lane l holds chunk l)
  float lo = INFINITY, hi = -INFINITY, badf = 0.f;
  if (lane < S.n_chunks) {
    const float4 p = S.part[lane];
    lo = p.x; hi = p.y; badf = p.z;
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    badf = fmaxf(badf, __shfl_xor(badf, o, 64));
  }
  __syncthreads();                                  // c64 ready
  const int strips_x = (S.cols + DCT_STRIP - 1) / DCT_STRIP;
  const int R0 = (lid / strips_x) * 16;
  const int CW = (lid % strips_x) * DCT_STRIP + wave * 64;   // this wave's 16 x 64 sub-strip
  if (lid == 0 && tid == 0 && S.lohi) { S.lohi[0] = lo; S.lohi[1] = hi; }
  const int j = lane & 15, g = lane >> 4;
  if (badf != 0.f || hi == lo) {     // constant or non-finite segment: sent as is, codes 0
    for (int r = 0; r < 16; ++r) {
      const int row = R0 + r, col = CW + lane;
      if (row < S.rows && col < S.cols && col < CW + 64) {
        if (S.dst != S.src) S.dst[(size_t)row * S.ld + col] = S.src[(size_t)row * S.ld + col];
        if (S.coeffs) S.coeffs[(size_t)row * S.cols + col] = 0;
      }
    }
    return;
  }
  // constant operands: forward B = C2^T, inverse B = C2 (lane j + 16g, step s -> row 4g + s)
  float Bf[4], Bi[4], qs[4];
  const int scale = quality < 50 ? 5000 / quality : 200 - 2 * quality;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = 4 * g + s;
    const bool same = (k >> 3) == (j >> 3);
    Bf[s] = same ? (float)c64[(j & 7) * 8 + (k & 7)] : 0.f;    // C2^T[k][j] = C2[j][k]
    Bi[s] = same ? (float)c64[(k & 7) * 8 + (j & 7)] : 0.f;    // C2[k][j]
    const int t = (int)kLumaTable[(k & 7) * 8 + (j & 7)];     // block position (row k%8, col j%8)
    qs[s] = (float)min(255, max(1, (t * scale + 50) / 100));
  }
  const float mapm = 255.f / (hi - lo);
  const float unm = (hi - lo) / 255.f;
  const double lo64 = lo, span64 = (double)hi - (double)lo;
  const float* src = S.src;
  // the wave's four tiles: all loads issued first
  f4 X[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = CW + 16 * t + j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = R0 + 4 * g + r;
      X[t][r] = (row < S.rows && col < S.cols) ? src[(size_t)row * S.ld + col] : lo;
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int C0 = CW + 16 * t;
    if (C0 >= S.cols) break;                        // uniform across the wave
    const int col = C0 + j;
    f4 V;
#pragma unroll
    for (int r = 0; r < 4; ++r) V[r] = (X[t][r] - lo) * mapm - 128.f;
    const f4 D1 = mfma_chain(V, Bf);      // (C2 V)^T
    const f4 F = mfma_chain(D1, Bf);      // C2 V C2^T
    float qv[4];
    bool tie[4];
    bool any = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = R0 + 4 * g + r;
      const float step = qs[r];
      const float tq = F[r] / step;
      qv[r] = rintf(tq);
      const float fr = fabsf(tq - truncf(tq));
      tie[r] = row < S.rows && col < S.cols && fabsf(fr - 0.5f) * step < 2e-3f;
      any = any || tie[r];
    }
    if (__ballot(any)) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!tie[r]) continue;
        // coefficient (u, v) of the block whose top-left pixel is (br, bc)
        const int tr = 4 * g + r;
        const int u = tr & 7, v = j & 7;
        const int br = R0 + (tr & 8), bc = C0 + (j & 8);
        double f = 0.0;
        for (int y = 0; y < 8; ++y) {
          double rowsum = 0.0;
          const float* line = src + (size_t)(br + y) * S.ld + bc;
          for (int x = 0; x < 8; ++x) {
            const double lv = ((double)line[x] - lo64) * 255.0 / span64 - 128.0;
            rowsum += c64[v * 8 + x] * lv;
          }
          f += c64[u * 8 + y] * rowsum;
        }
        qv[r] = (float)rint(f / (double)qs[r]);
      }
    }
    f4 Fq;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = R0 + 4 * g + r;
      if (S.coeffs && row < S.rows && col < S.cols) S.coeffs[(size_t)row * S.cols + col] = (int16_t)qv[r];
      Fq[r] = qv[r] * qs[r];
    }
    const f4 D3 = mfma_chain(Fq, Bi);     // F^T C2
    const f4 R = mfma_chain(D3, Bi);      // C2^T F C2
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = R0 + 4 * g + r;
      if (row < S.rows && col < S.cols) S.dst[(size_t)row * S.ld + col] = (R[r] + 128.f) * unm + lo;
    }
  }
}

// ---------------------------------------------------------------------------
// Segment x-update without a quantizer (or the averaged segment copied out)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_seg_none(const SegJob* jobs, int do_x, int e2) {
  const SegJob S = jobs[blockIdx.x];
  if (do_x) {
    segment_xupdate<256>(S, e2, S.xt);
  } else if (S.xt) {     // the averaged segment, copied out
    const size_t base = (size_t)S.row0 * S.n, cnt = (size_t)S.rows * S.n;
    for (size_t i = threadIdx.x; i < cnt; i += 256) S.xt[i] = S.x[base + i];
  }
}

// Eq. 9: x = mean over the slice's nodes of (u_m + lambda_m / rho); one job per
// slice.  With a regularization block, the closed-form argmin with its term:
// (sum_m rho_m (u_m + lambda_m / rho_m) + rho_z t_z) / (sum_m rho_m + rho_z).
__global__ __launch_bounds__(256) void k_avg(Many<AvgJob> src, const NodeRef* nodes) {
  int lid;
  const AvgJob A = src.get(blockIdx.x, lid);
  const size_t i = (size_t)lid * 256 + threadIdx.x;
  const size_t cnt = (size_t)A.n * A.n;
  if (i >= cnt) return;
  float s = 0.f;
  if (A.tz) {
    float w = A.rho_z;
    s = A.rho_z * A.tz[i];
    for (int m = 0; m < A.n_nodes; ++m) {
      const NodeRef R = nodes[A.node0 + m];
      s += R.rho * (R.u[i] + R.lam[i] / R.rho);
      w += R.rho;
    }
    A.x[i] = s / w;
    return;
  }
  for (int m = 0; m < A.n_nodes; ++m) {
    const NodeRef R = nodes[A.node0 + m];
    s += R.u[i] + R.lam[i] / R.rho;
  }
  A.x[i] = s / (float)A.n_nodes;
}

// Eq. 24 for every node: lambda_m += rho (u_m - x); four values per thread,
// as float4 when the three images are 16-byte aligned
__global__ __launch_bounds__(256) void k_dual(Many<NodeRef> src) {
  int lid;
  const NodeRef R = src.get(blockIdx.x, lid);
  const size_t cnt = (size_t)R.n * R.n;
  const size_t i0 = ((size_t)lid * 256 + threadIdx.x) * 4;
  if (i0 >= cnt) return;
  const bool vec = ((reinterpret_cast<uintptr_t>(R.u) | reinterpret_cast<uintptr_t>(R.x) |
                     reinterpret_cast<uintptr_t>(R.lam)) & 15) == 0;
  if (vec && i0 + 4 <= cnt) {
    const float4 u = *reinterpret_cast<const float4*>(R.u + i0);
    const float4 x = *reinterpret_cast<const float4*>(R.x + i0);
    float4 l = *reinterpret_cast<const float4*>(R.lam + i0);
    l.x = fmaf(R.rho, u.x - x.x, l.x);
    l.y = fmaf(R.rho, u.y - x.y, l.y);
    l.z = fmaf(R.rho, u.z - x.z, l.z);
    l.w = fmaf(R.rho, u.w - x.w, l.w);
    *reinterpret_cast<float4*>(R.lam + i0) = l;
  } else {
    for (size_t i = i0; i < cnt && i < i0 + 4; ++i) R.lam[i] = fmaf(R.rho, R.u[i] - R.x[i], R.lam[i]);
  }
}

// sum of squared differences in float64 (one workgroup, fixed reduction order)
__global__ __launch_bounds__(1024) void k_sqdiff(const float* a, const float* b, long long n,
                                                double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += 1024) {
    double d = (double)a[i] - (double)b[i];
    s += d * d;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += red[i];
    out[0] = t;
  }
}

}  // namespace tomo
