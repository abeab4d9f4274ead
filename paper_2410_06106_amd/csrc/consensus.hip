// Consensus, exchange and dual steps of decentralized ADMM (gfx950):
//   Alg. 3   segment x-update, E2 gradient steps on rho/2 ||u - x + lambda/rho||^2
//   Eq. 9    averaging x-update x = mean_m (u_m + lambda_m / rho)
//   Sec. 2.7 JPEG-style quantizer: 8x8 DCT-II on MFMA, table quantization, inverse DCT
//   Eq. 24   dual update lambda_m += rho (u_m - x)
// The x-update without a quantizer runs one workgroup per segment; with the DCT
// quantizer it is fused into the first of the codec's two many-workgroup
// launches.  (The K-means quantizer lives in kmeans.hip.)
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
  const float q = S.tz ? xseg_c(S.rho, S.rho_z, S.eta2, e2) : xseg_q(S.rho, S.eta2, e2);
  for (size_t i = threadIdx.x; i < cnt; i += NT) {
    float xv = S.x[base + i];
    const float tm = reg_target(S.u[base + i], S.lam[base + i], irho);
    if (e2 > 0) xv = S.tz ? xseg_reg(xv, tm, S.tz[base + i], S.rho, S.rho_z, q) : xseg(xv, tm, q);
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
// block-diagonal matrix C2 = diag(C, C): with a matrix Y held in the
// accumulator layout of v_mfma_f32_16x16x4_f32 (lane j + 16 g, register r holds
// Y[4g + r][j]) and passed as the A operand, one 4-instruction chain computes
// Y^T B; two chains transform a tile forward, two more back.
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

// A copy of the job owning workgroup bid of a launch (jobs == null: the
// launch has the one job `single`).  With uni > 0 every job spans uni
// workgroups and the index is bid / uni; otherwise it is found by the
// first-workgroup field F.  The table is read through the constant address
// space (scalar loads), and a copy cannot alias the arrays the kernel writes.
template <int SegJob::*F>
__device__ __forceinline__ SegJob job_of(const SegJob* jobs, int n_jobs, int uni, const SegJob& single, int bid) {
  if (!jobs) return single;
  const auto J = (const __attribute__((address_space(4))) SegJob*)jobs;
  int lo = 0, hi = n_jobs - 1;
  if (uni > 0) {
    lo = bid / uni;
  } else {
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (J[mid].*F <= bid) lo = mid; else hi = mid - 1;
    }
  }
  static_assert(sizeof(SegJob) % 4 == 0, "descriptor copied in 32-bit words");
  SegJob r;
  const auto w = (const __attribute__((address_space(4))) int*)(J + lo);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(SegJob) / 4); ++i) reinterpret_cast<int*>(&r)[i] = w[i];
  return r;
}

// global-address-space views (global loads and stores instead of flat ones)
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gas(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__global__ __launch_bounds__(DCT_THREADS) void k_dct_range(const SegJob* jobs, int n_jobs, int uni, SegJob single,
                                                           int do_x, int e2) {
  __shared__ float red[2 * (DCT_THREADS / 64)];
  __shared__ int redb[DCT_THREADS / 64];
  const SegJob S = job_of<&SegJob::range_wg>(jobs, n_jobs, uni, single, blockIdx.x);
  const int chunk = blockIdx.x - S.range_wg;
  const int r0 = chunk * S.chunk_rows, r1 = min(S.rows, r0 + S.chunk_rows);
  const int tid = threadIdx.x;
  const float irho = 1.f / S.rho;
  // row pieces of four values move as float4 when every array allows it
  auto al16 = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 15) == 0; };
  const bool vec = (S.cols & 3) == 0 && (S.ld & 3) == 0 && al16(S.src) && (!S.xt || al16(S.xt)) &&
                   (!do_x || (al16(S.x) && al16(S.u) && al16(S.lam) && (!S.tz || al16(S.tz)) && (S.n & 3) == 0));
  float lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  const float xq = S.tz ? xseg_c(S.rho, S.rho_z, S.eta2, e2) : xseg_q(S.rho, S.eta2, e2);
  auto update = [&](float v, size_t i) {   // Alg. 3 on value v of x at index i of the slice
    const float tm = reg_target(S.u[i], S.lam[i], irho);
    if (e2 > 0) v = S.tz ? xseg_reg(v, tm, S.tz[i], S.rho, S.rho_z, xq) : xseg(v, tm, xq);
    return v;
  };
  auto fold = [&](float v) {
    bad |= !isfinite(v);
    lo = fminf(lo, v);
    hi = fmaxf(hi, v);
  };
  if (vec) {
    // the chunk's float4s, DCT_VEC per thread and pass, every load of a pass
    // issued before any is used
    constexpr int DCT_VEC = 4;
    const int per_row = S.cols >> 2;
    const int total = (r1 - r0) * per_row;
    for (int base = 0; base < total; base += DCT_THREADS * DCT_VEC) {
      f4 a[DCT_VEC], uu[DCT_VEC], ll[DCT_VEC], tt[DCT_VEC];
      size_t ix[DCT_VEC];
      bool ok[DCT_VEC];
#pragma unroll
      for (int q = 0; q < DCT_VEC; ++q) {
        const int f = base + q * DCT_THREADS + tid;
        ok[q] = f < total;
        const int ff = ok[q] ? f : total - 1;
        const int r = r0 + ff / per_row, c = 4 * (ff - (ff / per_row) * per_row);
        if (do_x) {       // consensus: the segment of x, ld = cols = n
          ix[q] = (size_t)(S.row0 + r) * S.n + c;
          a[q] = *(const __attribute__((address_space(1))) f4*)gas(S.x + ix[q]);
          uu[q] = *(const __attribute__((address_space(1))) f4*)gas(S.u + ix[q]);
          ll[q] = *(const __attribute__((address_space(1))) f4*)gas(S.lam + ix[q]);
          if (S.tz) tt[q] = *(const __attribute__((address_space(1))) f4*)gas(S.tz + ix[q]);
        } else {
          ix[q] = (size_t)r * S.ld + c;
          a[q] = *(const __attribute__((address_space(1))) f4*)gas(S.src + ix[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < DCT_VEC; ++q) {
        if (do_x) {
          float* v = reinterpret_cast<float*>(&a[q]);
          const float* uv = reinterpret_cast<const float*>(&uu[q]);
          const float* lv = reinterpret_cast<const float*>(&ll[q]);
          const float* tv = reinterpret_cast<const float*>(&tt[q]);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float tm = reg_target(uv[c], lv[c], irho);
            if (e2 > 0) v[c] = S.tz ? xseg_reg(v[c], tm, tv[c], S.rho, S.rho_z, xq) : xseg(v[c], tm, xq);
          }
          if (ok[q]) *(__attribute__((address_space(1))) f4*)gas(S.x + ix[q]) = a[q];
        }
        if (ok[q]) {
          if (S.xt) {
            const int f = base + q * DCT_THREADS + tid;
            *(__attribute__((address_space(1))) f4*)gas(S.xt + (size_t)(r0 + f / per_row) * S.cols +
                                                      4 * (f - (f / per_row) * per_row)) = a[q];
          }
          fold(a[q][0]);
          fold(a[q][1]);
          fold(a[q][2]);
          fold(a[q][3]);
        }
      }
    }
  } else {
    for (int r = r0; r < r1; ++r) {
      for (int c = tid; c < S.cols; c += DCT_THREADS) {
        float v;
        if (do_x) {
          const size_t i = (size_t)(S.row0 + r) * S.n + c;
          v = update(S.x[i], i);
          S.x[i] = v;
        } else {
          v = S.src[(size_t)r * S.ld + c];
        }
        if (S.xt) S.xt[(size_t)r * S.cols + c] = v;
        fold(v);
      }
    }
  }
  wg_minmax<DCT_THREADS>(lo, hi, bad, red, redb);
  if (tid == 0) S.part[chunk] = make_float4(lo, hi, bad ? 1.f : 0.f, 0.f);
}

// Coding.  The wave holds each 16x16 tile transposed: lane j + 16 g, register r
// holds X[j][4g + r] (one row piece of four values, a float4 when aligned), i.e.
// Y = X^T in the accumulator layout; the forward chains then give F^T, so the
// lane's register r holds the coefficient of tile row j, tile column 4g + r
// (block row j / 8, vertical frequency j % 8; block column (4g + r) / 8,
// horizontal frequency (4g + r) % 8), and the inverse chains give the decoded
// tile in the same layout: codes and decoded values are stored as row pieces too.
// (at most 128 VGPRs: four waves per SIMD, so a launch of four workgroups per
// CU runs in one round)
__global__ __launch_bounds__(DCT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void k_dct_code(const SegJob* jobs, int n_jobs, int uni, SegJob single, int quality) {
  __shared__ double c64[64];
  __shared__ double tile_s[DCT_THREADS / 64][16 * 17];  // a wave's level-mapped tile, for ties
  const SegJob S = job_of<&SegJob::code_wg>(jobs, n_jobs, uni, single, blockIdx.x);
  const int lid = blockIdx.x - S.code_wg;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int strips_x = (S.cols + DCT_STRIP - 1) / DCT_STRIP;
  const int R0 = (lid / strips_x) * 16;
  const int CW = (lid % strips_x) * DCT_STRIP + wave * 64;   // this wave's 16 x 64 sub-strip
  const int row = R0 + j;
  const bool vec = (S.cols & 3) == 0 && (S.ld & 3) == 0 && ((reinterpret_cast<uintptr_t>(S.src) |
                   reinterpret_cast<uintptr_t>(S.dst)) & 15) == 0;
  const bool vcode = S.coeffs && (reinterpret_cast<uintptr_t>(S.coeffs) & 7) == 0;
  // the wave's four tiles, loaded first (in flight while the tables are set up)
  f4 X[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int col = CW + 16 * t + 4 * g;             // col..col+3 lie in range together (cols % 8 == 0)
    if (row < S.rows && col < S.cols) {
      const auto q = gas(S.src + (size_t)row * S.ld + col);
      if (vec) {
        X[t] = *(const __attribute__((address_space(1))) f4*)q;
      } else {
        X[t][0] = q[0]; X[t][1] = q[1]; X[t][2] = q[2]; X[t][3] = q[3];
      }
    } else {
      X[t][0] = X[t][1] = X[t][2] = X[t][3] = 0.f;
    }
  }
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
  if (lid == 0 && tid == 0 && S.lohi) { S.lohi[0] = lo; S.lohi[1] = hi; }
  if (badf != 0.f || hi == lo) {     // constant or non-finite segment: sent as is, codes 0
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = CW + 16 * t + 4 * g;
      if (row < S.rows && col < S.cols) {
        for (int c = 0; c < 4; ++c) {
          if (S.dst != S.src) S.dst[(size_t)row * S.ld + col + c] = X[t][c];
          if (S.coeffs) S.coeffs[(size_t)row * S.cols + col + c] = 0;
        }
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
    // the step of this lane's coefficient r = s: vertical frequency j % 8,
    // horizontal frequency (4g + s) % 8
    const int tq = (int)kLumaTable[(j & 7) * 8 + (k & 7)];
    qs[s] = (float)min(255, max(1, (tq * scale + 50) / 100));
  }
  const float mapm = 255.f / (hi - lo);
  const float unm = (hi - lo) / 255.f;
  const double lo64 = lo, span64 = (double)hi - (double)lo;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int C0 = CW + 16 * t;
    if (C0 >= S.cols) break;                        // uniform across the wave
    const int col = C0 + 4 * g;
    const bool in = row < S.rows && col < S.cols;
    f4 V;
#pragma unroll
    for (int r = 0; r < 4; ++r) V[r] = in ? (X[t][r] - lo) * mapm - 128.f : 0.f;
    const f4 D1 = mfma_chain(V, Bf);      // X C2^T
    const f4 F = mfma_chain(D1, Bf);      // (C2 X C2^T)^T
    float qv[4];
    bool tie[4];
    bool any = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float step = qs[r];
      const float tq = F[r] / step;
      qv[r] = rintf(tq);
      const float fr = fabsf(tq - truncf(tq));
      tie[r] = in && fabsf(fr - 0.5f) * step < 2e-3f;
      any = any || tie[r];
    }
    if (__ballot(any)) {
      // every lane of the wave is here (the branch is uniform): the tile's
      // level-mapped values in float64 go to the wave's LDS slot (row j,
      // columns 4g..4g+3; blocks lie wholly inside the segment), one division
      // per value, and the lanes at a tie read their block from there
      double* tl = tile_s[wave];
#pragma unroll
      for (int r = 0; r < 4; ++r) tl[j * 17 + 4 * g + r] = ((double)X[t][r] - lo64) * 255.0 / span64 - 128.0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!tie[r]) continue;
        // coefficient (u, v) of the 8x8 block at tile offset (br, bc)
        const int u = j & 7, v = (4 * g + r) & 7;
        const double* blk = tl + (j & 8) * 17 + ((4 * g + r) & 8);
        double f = 0.0;
        for (int y = 0; y < 8; ++y) {
          double rowsum = 0.0;
#pragma unroll
          for (int x = 0; x < 8; ++x) rowsum += c64[v * 8 + x] * blk[y * 17 + x];
          f += c64[u * 8 + y] * rowsum;
        }
        qv[r] = (float)rint(f / (double)qs[r]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // reads done before the slot is reused
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    f4 Fq;
#pragma unroll
    for (int r = 0; r < 4; ++r) Fq[r] = qv[r] * qs[r];
    if (S.coeffs && in) {
      const auto cq = gas(S.coeffs + (size_t)row * S.cols + col);
      if (vcode) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        u2 w;
        w[0] = (unsigned)(uint16_t)(int16_t)qv[0] | ((unsigned)(uint16_t)(int16_t)qv[1] << 16);
        w[1] = (unsigned)(uint16_t)(int16_t)qv[2] | ((unsigned)(uint16_t)(int16_t)qv[3] << 16);
        *(__attribute__((address_space(1))) u2*)cq = w;
      } else {
        for (int r = 0; r < 4; ++r) cq[r] = (int16_t)qv[r];
      }
    }
    const f4 D3 = mfma_chain(Fq, Bi);     // F C2
    const f4 R = mfma_chain(D3, Bi);      // (C2^T F C2)^T
    if (in) {
      f4 o;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = (R[r] + 128.f) * unm + lo;
      const auto q = gas(S.dst + (size_t)row * S.ld + col);
      if (vec) {
        *(__attribute__((address_space(1))) f4*)q = o;
      } else {
        q[0] = o[0]; q[1] = o[1]; q[2] = o[2]; q[3] = o[3];
      }
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
