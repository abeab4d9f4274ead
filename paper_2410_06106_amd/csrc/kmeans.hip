// Scalar K-means quantizer (Alg. 5) of exchanged segments, for gfx950.
//
// Arithmetic is fixed so that results are bit-exact and independent of the
// launch shape: centres start at lo + (hi - lo)(2j + 1)/(2k) (float64, no
// contraction); with the centres in increasing order a value's label is the
// number of midpoints below it, label(a) = #{j < k-1 : 2a > c_j + c_{j+1}}
// (float64: 2a exact, the sum rounded once), i.e. its nearest centre; values
// enter the centroid sums as fixed point q = round(a * 2^S), S = 30 - e (e the
// binary exponent of max(|lo|, |hi|), so |q| <= 2^30 fits an int32 and a * 2^S
// is exact in float32), summed in int64, so every sum is exact in any order; a
// centre becomes f32(f64(sum) * 2^-S / f64(count)) (empty clusters keep
// theirs), after which the centres are stably sorted; Lloyd iterations stop
// when no label changes or after max_iter.
//
// Because the label is monotone in the value, every cluster is a run of the
// sorted values, and the labelling is fixed by k - 1 boundary counts (values
// at or below each midpoint).  One workgroup owns a segment.  It buckets the
// values once by value range (a monotone bucket function), keeping exclusive
// prefix counts and exact int64 prefix sums of the codes per bucket, and
// regroups the values by bucket (in LDS, or in a global workspace for long
// segments).  The count and code sum at or below a midpoint are then the prefix
// of the buckets left of the midpoint's bucket plus that one bucket's share,
// found by a wave scanning it: a Lloyd iteration costs k - 1 bucket scans
// instead of a pass over every value, and "no label changed" is "no boundary
// count changed".  Labels and quantized values are written once at the end.
// The optional Alg. 3 x-update of the segment is applied on load.
#include "common.h"

namespace tomo {

namespace {

constexpr int KT = 1024;                // threads per workgroup
constexpr int KWAVES = KT / 64;
constexpr int KBUCKETS = 2048;          // value-range buckets at most
constexpr int KPER = KBUCKETS / KT;     // bucket entries per thread in the scan

struct KMShared {
  int start[KBUCKETS + 1];        // bucket counts, then their exclusive prefix (start[B] = n)
  int fill[KBUCKETS];             // values placed per bucket so far
  long long psum[KBUCKETS + 1];   // code sums per bucket, then their exclusive prefix
  double mid[KM_MAX_K];           // c_j + c_{j+1}
  float cent[KM_MAX_K];           // centres, increasing
  float upd[KM_MAX_K];            // updated centres before sorting
  int cb[2][KM_MAX_K + 1];        // values at or below midpoint j-1 (label < j), two generations
  long long sb[KM_MAX_K + 1];     // their code sums
  int wcnt[KWAVES];
  long long wsum[KWAVES];
  float red[2 * KWAVES];
  int redb[KWAVES];
};

__device__ __forceinline__ int km_fixed(float v, int S) {
  return (int)rintf(ldexpf(v, S));     // exact scaling, round half to even
}

__device__ __forceinline__ float km_xupdate(float xv, float uv, float lv, float rho, float irho, float eta2,
                                            int e2) {
  for (int e = 0; e < e2; ++e) {
    float delta = rho * (xv - uv - lv * irho);
    xv = xv - eta2 * delta;
  }
  return xv;
}

// Largest float32 below a finite x.
__device__ __forceinline__ float prev_float(float x) {
  if (x == 0.f) return __uint_as_float(0x80000001u);
  const unsigned u = __float_as_uint(x);
  return __uint_as_float(x > 0.f ? u - 1u : u + 1u);
}

// Monotone (non-decreasing) bucket index of a value a >= lo: every rounding
// step is monotone, so a < b implies bucket(a) <= bucket(b).
struct Buckets {
  float lo, scl, top;
  __device__ __forceinline__ int of(float a) const { return (int)fminf((a - lo) * scl, top); }
};

// Global-address-space views of a job's arrays (plain global loads and stores
// instead of flat accesses).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Exclusive prefix of the B bucket counts and code sums, in place; entry B
// receives the totals.
__device__ void bucket_scan(KMShared& sh, int B) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  int c[KPER];
  long long s[KPER];
  int ct = 0;
  long long st = 0;
#pragma unroll
  for (int r = 0; r < KPER; ++r) {
    const int b = tid * KPER + r;
    c[r] = b < B ? sh.start[b] : 0;
    s[r] = b < B ? sh.psum[b] : 0;
    ct += c[r];
    st += s[r];
  }
  int ic = ct;
  long long is = st;
  for (int o = 1; o < 64; o <<= 1) {
    const int oc = __shfl_up(ic, o, 64);
    const long long os = __shfl_up(is, o, 64);
    if (l >= o) { ic += oc; is += os; }
  }
  if (l == 63) { sh.wcnt[w] = ic; sh.wsum[w] = is; }
  __syncthreads();
  int ec = ic - ct;
  long long es = is - st;
  for (int q = 0; q < w; ++q) { ec += sh.wcnt[q]; es += sh.wsum[q]; }
#pragma unroll
  for (int r = 0; r < KPER; ++r) {
    const int b = tid * KPER + r;
    if (b < B) { sh.start[b] = ec; sh.psum[b] = es; }
    ec += c[r];
    es += s[r];
  }
  if (tid == KT - 1) { sh.start[B] = ec; sh.psum[B] = es; }
  __syncthreads();
}

// Count and code sum of the values with 2a <= m, for one wave (every lane
// gets the result).  Buckets left of the bucket of x = the largest float32 with
// 2x <= m hold only such values, buckets right of it none.
template <class VP>
__device__ __forceinline__ void at_or_below(const KMShared& sh, VP V, double m, const Buckets& bk, float lo,
                                            float hi, int n, long long tot, int S, int& cnt, long long& sum) {
  const double h = 0.5 * m;            // exact
  if (h < (double)lo) { cnt = 0; sum = 0; return; }
  if (h >= (double)hi) { cnt = n; sum = tot; return; }
  float x = (float)h;
  if ((double)x > h) x = prev_float(x);
  const int b = bk.of(x);
  const int p0 = sh.start[b], p1 = sh.start[b + 1];
  int c = 0;
  long long s = 0;
  for (int p = p0 + (int)(threadIdx.x & 63); p < p1; p += 64) {
    const float a = V[p];
    if (2.0 * (double)a <= m) { ++c; s += km_fixed(a, S); }
  }
  for (int o = 32; o > 0; o >>= 1) {
    c += __shfl_xor(c, o, 64);
    s += __shfl_xor(s, o, 64);
  }
  cnt = p0 + c;
  sum = sh.psum[b] + s;
}

}  // namespace

// One workgroup per segment.  VLDS: the bucket-ordered values fit in LDS
// (n <= KM_LDS_VALUES); otherwise they go to work + segment * work_stride.
template <bool VLDS>
__global__ __launch_bounds__(KT) void k_kmeans(const KMJob* jobs, KMJob single, int k, int max_iter, int e2,
                                               float* work, long long work_stride) {
#pragma clang fp contract(off)
  __shared__ KMShared sh;
  __shared__ float vlds[VLDS ? KM_LDS_VALUES : 1];
  const int seg = blockIdx.x;
  const KMJob J = jobs ? jobs[seg] : single;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int n = (int)J.n;
  const bool do_x = J.u != nullptr;
  const float irho = 1.f / J.rho;
  const auto src = gptr(J.src);
  const auto xo = gptr(J.x);
  const auto ahat = gptr(J.a_hat);
  const auto uu = gptr(J.u);
  const auto ll = gptr(J.lam);
  const auto labels = gptr(J.labels);
  const auto vals = do_x ? gptr((const float*)J.x) : src;   // the segment after the x-update
  if (n <= 0) {
    if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = 0.f;
    if (J.iters && tid == 0) *J.iters = 0;
    return;
  }

  // pass 1: x-update, range, finiteness
  float lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (int i = tid; i < n; i += KT) {
    float a = src[i];
    if (do_x) {
      a = km_xupdate(a, uu[i], ll[i], J.rho, irho, J.eta2, e2);
      xo[i] = a;
    }
    bad |= !isfinite(a);
    lo = fminf(lo, a);
    hi = fmaxf(hi, a);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  if (l == 0) { sh.red[2 * w] = lo; sh.red[2 * w + 1] = hi; sh.redb[w] = bad; }
  __syncthreads();
  lo = sh.red[0];
  hi = sh.red[1];
  bad = sh.redb[0];
  for (int q = 1; q < KWAVES; ++q) {
    lo = fminf(lo, sh.red[2 * q]);
    hi = fmaxf(hi, sh.red[2 * q + 1]);
    bad |= sh.redb[q];
  }
  if (bad || hi == lo) {
    // constant segment: one cluster at lo; non-finite input: flagged
    for (int i = tid; i < n; i += KT) {
      if (J.labels) labels[i] = 0;
      if (J.a_hat && J.a_hat != (do_x ? J.x : J.src)) ahat[i] = vals[i];
    }
    if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = bad ? 0.f : lo;
    if (J.iters && tid == 0) *J.iters = bad ? -1 : 0;
    return;
  }
  int e;
  frexp(fmax(fabs((double)lo), fabs((double)hi)), &e);
  const int S = 30 - e;
  const int B = min(KBUCKETS, max(1, n / 4));
  const Buckets bk{lo, (float)B / (hi - lo), (float)(B - 1)};

  // pass 2: bucket counts and code sums
  for (int b = tid; b < B; b += KT) { sh.start[b] = 0; sh.fill[b] = 0; sh.psum[b] = 0; }
  if (tid < k) {
    double lo64 = lo, hi64 = hi;
    double t = (hi64 - lo64) * (double)(2 * tid + 1);
    t = t / (double)(2 * k);
    sh.cent[tid] = (float)(lo64 + t);
  }
  __syncthreads();
  for (int i = tid; i < n; i += KT) {
    const float a = vals[i];
    const int b = bk.of(a);
    atomicAdd(&sh.start[b], 1);
    atomicAdd((unsigned long long*)&sh.psum[b], (unsigned long long)(long long)km_fixed(a, S));
  }
  __syncthreads();
  bucket_scan(sh, B);
  const long long tot = sh.psum[B];

  // pass 3: values regrouped by bucket
  float* const wv = VLDS ? nullptr : work + (size_t)seg * work_stride;
  for (int i = tid; i < n; i += KT) {
    const float a = vals[i];
    const int b = bk.of(a);
    const int p = sh.start[b] + atomicAdd(&sh.fill[b], 1);
    if constexpr (VLDS) vlds[p] = a;
    else gptr(wv)[p] = a;
  }
  if (tid < k - 1) sh.mid[tid] = (double)sh.cent[tid] + (double)sh.cent[tid + 1];
  if (tid == 0) {
    sh.cb[0][0] = sh.cb[1][0] = 0;
    sh.cb[0][k] = sh.cb[1][k] = n;
    sh.sb[0] = 0;
    sh.sb[k] = tot;
  }
  __syncthreads();

  auto boundaries = [&](int gen) {
    for (int j = w; j < k - 1; j += KWAVES) {
      int c;
      long long s;
      if constexpr (VLDS) at_or_below(sh, vlds, sh.mid[j], bk, lo, hi, n, tot, S, c, s);
      else at_or_below(sh, gptr((const float*)wv), sh.mid[j], bk, lo, hi, n, tot, S, c, s);
      if (l == 0) { sh.cb[gen][j + 1] = c; sh.sb[j + 1] = s; }
    }
  };

  boundaries(0);
  __syncthreads();
  int cur = 0, it = 0;
  for (int t = 1; t <= max_iter; ++t) {
    if (tid < k) {
      const int c = sh.cb[cur][tid + 1] - sh.cb[cur][tid];
      float cj = sh.cent[tid];
      if (c > 0) cj = (float)(ldexp((double)(sh.sb[tid + 1] - sh.sb[tid]), -S) / (double)c);
      sh.upd[tid] = cj;
    }
    __syncthreads();
    if (tid < k) {                     // stable rank sort of the k centres
      const float cj = sh.upd[tid];
      int r = 0;
      for (int i = 0; i < k; ++i) {
        const float ci = sh.upd[i];
        r += (ci < cj) || (ci == cj && i < tid);
      }
      sh.cent[r] = cj;
    }
    __syncthreads();
    if (tid < k - 1) sh.mid[tid] = (double)sh.cent[tid] + (double)sh.cent[tid + 1];
    __syncthreads();
    boundaries(cur ^ 1);
    __syncthreads();
    it = t;
    const int moved = tid <= k && sh.cb[cur ^ 1][tid] != sh.cb[cur][tid];
    cur ^= 1;
    if (!__syncthreads_or(moved)) break;
  }

  // labels and quantized values: the count of midpoints below 2a
  for (int i = tid; i < n; i += KT) {
    const float a = vals[i];
    const double t2 = 2.0 * (double)a;
    int p = 0, len = k - 1;
    while (len > 0) {
      const int half = len >> 1;
      if (sh.mid[p + half] < t2) { p += half + 1; len -= half + 1; }
      else len = half;
    }
    if (J.labels) labels[i] = (uint8_t)p;
    if (J.a_hat) ahat[i] = sh.cent[p];
  }
  if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = sh.cent[j];
  if (J.iters && tid == 0) *J.iters = it;
}

template __global__ void k_kmeans<true>(const KMJob*, KMJob, int, int, int, float*, long long);
template __global__ void k_kmeans<false>(const KMJob*, KMJob, int, int, int, float*, long long);

}  // namespace tomo
