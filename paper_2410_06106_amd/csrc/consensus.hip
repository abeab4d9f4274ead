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
template <int NT>
__device__ void segment_xupdate(const SegJob& S, int e2) {
  const size_t base = (size_t)S.row0 * S.n;
  const size_t cnt = (size_t)S.rows * S.n;
  const float irho = 1.f / S.rho;
  for (size_t i = threadIdx.x; i < cnt; i += NT) {
    float xv = S.x[base + i];
    const float uv = S.u[base + i], lv = S.lam[base + i];
    if (S.tz) {
      const float tm = reg_target(uv, lv, irho), tv = S.tz[base + i];
      for (int e = 0; e < e2; ++e) xv = xstep_reg(xv, tm, tv, S.rho, S.rho_z, S.eta2);
    } else {
      for (int e = 0; e < e2; ++e) {
        float delta = S.rho * (xv - uv - lv * irho);
        xv = xv - S.eta2 * delta;
      }
    }
    S.x[base + i] = xv;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// JPEG-style codec on MFMA.  A wave transforms one 16x16 tile = 2x2 blocks at
// a time with the block-diagonal matrix C2 = diag(C, C).  With the tile X held
// in the accumulator layout of v_mfma_f32_16x16x4_f32 (lane j + 16 g, register
// r holds X[4g + r][j]) and passed as the A operand, one 4-instruction chain
// computes X^T B; two chains give C2 V C2^T forward and C2^T F C2 inverse.
// ---------------------------------------------------------------------------
constexpr int DCT_THREADS = 256;
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

__device__ __forceinline__ float dct_coef(int u, int x) {   // C[u][x], orthonormal DCT-II
  double al = u == 0 ? sqrt(0.125) : 0.5;
  return (float)(al * cos((2 * x + 1) * u * 3.14159265358979323846 / 16.0));
}

__device__ __forceinline__ f4 mfma_chain(const f4& X, const float* B) {
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[0], B[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[1], B[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[2], B[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(X[3], B[3], acc, 0, 0, 0);
  return acc;
}

struct DCTShared {
  float red[2 * (DCT_THREADS / 64)];
  int redb[DCT_THREADS / 64];
};

__device__ void dct_wg(const float* a, int rows, int cols, int ld, int quality, int16_t* coeffs,
                       float* a_hat, float* lohi, DCTShared& sh) {
  const int tid = threadIdx.x;
  float lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int r = 0; r < rows; ++r)
    for (int c = tid; c < cols; c += DCT_THREADS) {
      float v = a[(size_t)r * ld + c];
      bad |= !isfinite(v);
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
  wg_minmax<DCT_THREADS>(lo, hi, bad, sh.red, sh.redb);
  if (lohi && tid == 0) { lohi[0] = lo; lohi[1] = hi; }
  if (bad || hi == lo) {
    for (int r = 0; r < rows; ++r)
      for (int c = tid; c < cols; c += DCT_THREADS) {
        if (a_hat && a_hat != a) a_hat[(size_t)r * ld + c] = a[(size_t)r * ld + c];
        if (coeffs) coeffs[(size_t)r * cols + c] = 0;
      }
    return;
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int j = lane & 15, g = lane >> 4;
  // constant operands: forward B = C2^T, inverse B = C2 (lane j + 16g, step s -> row 4g + s)
  float Bf[4], Bi[4], qs[4];
  const int scale = quality < 50 ? 5000 / quality : 200 - 2 * quality;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int k = 4 * g + s;
    bool same = (k >> 3) == (j >> 3);
    Bf[s] = same ? dct_coef(j & 7, k & 7) : 0.f;      // C2^T[k][j] = C2[j][k]
    Bi[s] = same ? dct_coef(k & 7, j & 7) : 0.f;      // C2[k][j]
    int t = (int)kLumaTable[(k & 7) * 8 + (j & 7)];   // block position (row k%8, col j%8)
    qs[s] = (float)min(255, max(1, (t * scale + 50) / 100));
  }
  const float mapm = 255.f / (hi - lo);
  const float unm = (hi - lo) / 255.f;
  const int tr = (rows + 15) / 16, tc = (cols + 15) / 16;
  for (int tile = wave; tile < tr * tc; tile += DCT_THREADS / 64) {
    const int R0 = (tile / tc) * 16, C0 = (tile % tc) * 16;
    const int col = C0 + j;
    f4 X;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = R0 + 4 * g + r;
      float v = 0.f;
      if (row < rows && col < cols) v = (a[(size_t)row * ld + col] - lo) * mapm - 128.f;
      X[r] = v;
    }
    f4 D1 = mfma_chain(X, Bf);        // (C2 V)^T
    f4 F = mfma_chain(D1, Bf);        // C2 V C2^T
    f4 Fq;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // row 4g + r of the tile: block row (4g + r) % 8 = its quant-table row
      const float step = qs[r];
      float qv = rintf(F[r] / step);
      int row = R0 + 4 * g + r;
      if (coeffs && row < rows && col < cols) coeffs[(size_t)row * cols + col] = (int16_t)qv;
      Fq[r] = qv * step;
    }
    f4 D3 = mfma_chain(Fq, Bi);       // F^T C2
    f4 V = mfma_chain(D3, Bi);        // C2^T F C2
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = R0 + 4 * g + r;
      if (row < rows && col < cols) a_hat[(size_t)row * ld + col] = (V[r] + 128.f) * unm + lo;
    }
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_seg_none(const SegJob* jobs, int do_x, int e2) {
  const SegJob S = jobs[blockIdx.x];
  if (do_x) segment_xupdate<256>(S, e2);
}

__global__ __launch_bounds__(DCT_THREADS) void k_seg_dct(const SegJob* jobs, int do_x, int e2,
                                                         int quality) {
  __shared__ DCTShared sh;
  const SegJob S = jobs[blockIdx.x];
  if (do_x) segment_xupdate<DCT_THREADS>(S, e2);
  float* seg = S.x + (size_t)S.row0 * S.n;
  dct_wg(seg, S.rows, S.n, S.n, quality, S.coeffs, seg, S.lohi, sh);
}

__global__ __launch_bounds__(DCT_THREADS) void k_dct(const float* a, int rows, int cols, int ld,
                                                    int quality, int16_t* coeffs, float* a_hat,
                                                    float* lohi) {
  __shared__ DCTShared sh;
  dct_wg(a, rows, cols, ld, quality, coeffs, a_hat, lohi, sh);
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
