// Scalar K-means quantizer (Alg. 5) of exchanged segments, for gfx950.
//
// Arithmetic is fixed so that results are bit-exact and independent of the
// launch shape: centres start at lo + (hi - lo)(2j + 1)/(2k) (float64, no
// contraction); values enter the centroid sums as fixed point
// q = round(a * 2^S), S = 30 - e (e the binary exponent of max(|lo|, |hi|), so
// |q| <= 2^30 fits an int32 and a * 2^S is exact in float32), summed in int64,
// so every sum is exact in any order;
// label = lowest j minimising |a - c_j| in float32; a centre becomes
// f32(f64(sum) * 2^-S / f64(count)); Lloyd iterations stop when no label
// changes or after max_iter.
//
// One segment is spread over G workgroups (G * segments <= number of CUs, so
// all of them are resident together).  Each iteration a workgroup publishes the
// cluster sums of its slice of the segment to a double-buffered slot and meets
// the others at a per-segment barrier; every workgroup then adds the G slots in
// the same order and derives identical centres.  The barrier spins a bounded
// number of times: if the workgroups of a segment ever fail to be co-resident
// the kernel reports iters = -2 instead of hanging.  With G = 1 no barrier is
// needed.  The optional Alg. 3 x-update of the segment is applied on load.
#include "common.h"

namespace tomo {

namespace {

constexpr int KT = 1024;                // threads per workgroup
constexpr int KWAVES = KT / 64;
constexpr int KVPT = 16;                // values per thread kept in registers
constexpr int KCOPY = 4;                // replicas of each cluster bin (fewer LDS atomic conflicts)
constexpr unsigned kSpinLimit = 1u << 20;

__device__ __forceinline__ int km_assign(float v, const float* cent, int k) {
  float best = fabsf(v - cent[0]);
  int bj = 0;
  for (int j = 1; j < k; ++j) {
    float d = fabsf(v - cent[j]);
    if (d < best) { best = d; bj = j; }
  }
  return bj;
}

// Same result as km_assign when the centres are sorted (non-decreasing): with
// p the first centre >= v, |v - c_j| (float32) does not increase for j < p and
// does not decrease for j >= p, so the minimum is at p - 1 or p; ties go to the
// lowest index, found by walking left over equal distances.
__device__ __forceinline__ int km_assign_sorted(float v, const float* cent, int k, int steps) {
  int lo = 0, len = k;              // lower bound: p in [lo, lo + len]
  for (int s = 0; s < steps; ++s) {  // 2^steps > k, so len reaches 0
    int step = len >> 1;
    int mid = lo + step;             // < lo + len <= k whenever len > 0
    bool right = len > 0 && cent[mid] < v;
    lo = right ? mid + 1 : lo;
    len = right ? len - step - 1 : step;
  }
  const int p = lo;
  if (p == 0) return 0;
  const float dl = fabsf(v - cent[p - 1]);
  if (p < k && fabsf(v - cent[p]) < dl) return p;
  int j = p - 1;
  while (j > 0 && fabsf(v - cent[j - 1]) == dl) --j;
  return j;
}

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

constexpr int KMAXG = 16;               // workgroups per segment at most

struct KMLocal {
  unsigned long long sum[KWAVES][KM_MAX_K];   // per-wave cluster sums (KCOPY replicas when k <= 64)
  unsigned cnt[KWAVES][KM_MAX_K];
  long long gsum[KMAXG][KM_MAX_K];            // every workgroup's published sums of the segment
  unsigned gcnt[KMAXG][KM_MAX_K];
  float cent[KM_MAX_K];
  float red[2 * KWAVES];
  int redb[KWAVES];
  float gmn[KMAXG], gmx[KMAXG];
  int gflag[KMAXG];
  int flag;
  int ok;
  int sorted;
};

// Monotonic per-segment barrier: the b-th barrier of a launch completes when
// the arrival counter reaches b * G.  Returns false after kSpinLimit polls.
// Cross-workgroup data of a segment (the statistic slots and the barrier
// counter) is only ever accessed with device-scope atomic loads and stores,
// which are coherent across the XCDs without cache maintenance; a device-scope
// release or acquire fence would write back or invalidate a whole L2, which
// costs more than the Lloyd iteration itself.  Before arriving, every wave
// waits for its own slot stores to complete.
__device__ bool seg_barrier(KMSync* sy, int G, unsigned b, KMLocal& sh) {
  if (G == 1) {
    __syncthreads();
    return true;
  }
  __builtin_amdgcn_s_waitcnt(0);   // this wave's slot stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(&sy->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = b * (unsigned)G;
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(&sy->arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) { ok = 0; break; }
    }
    sh.ok = ok;
  }
  __syncthreads();
  return sh.ok != 0;
}

template <typename T>
__device__ __forceinline__ void put(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T get(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void seg_leave(KMSync* sy, int G) {
  __syncthreads();
  if (G == 1 || threadIdx.x != 0) return;
  // every workgroup has passed its last barrier: the last one out resets them
  if (__hip_atomic_fetch_add(&sy->leave, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)(G - 1)) {
    __hip_atomic_store(&sy->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&sy->leave, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}


}  // namespace

// Labels of KVPT register-resident values: the centres are read once each
// (outer loop) and compared with every value; sorted centres with k > 8 use
// the equivalent binary search.
template <int NV>
__device__ __forceinline__ void assign_regs(const float (&v)[NV], uint8_t (&lab)[NV], const float* cent, int k,
                                            int steps, int sorted) {
  if (k > 8 && sorted) {
#pragma unroll
    for (int q = 0; q < NV; ++q) lab[q] = (uint8_t)km_assign_sorted(v[q], cent, k, steps);
    return;
  }
  constexpr int H = NV > 8 ? 8 : NV;   // values per pass (bounds register use)
#pragma unroll
  for (int h0 = 0; h0 < NV; h0 += H) {
    float best[H];
    const float c0 = cent[0];
#pragma unroll
    for (int q = 0; q < H; ++q) { best[q] = fabsf(v[h0 + q] - c0); lab[h0 + q] = 0; }
    for (int j = 1; j < k; ++j) {
      const float c = cent[j];
#pragma unroll
      for (int q = 0; q < H; ++q) {
        float d = fabsf(v[h0 + q] - c);
        bool lt = d < best[q];
        best[q] = lt ? d : best[q];
        lab[h0 + q] = lt ? (uint8_t)j : lab[h0 + q];
      }
    }
  }
}

// Global-address-space views of a job's arrays (plain global loads and stores
// instead of flat accesses).
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

template <bool REG>
__global__ __launch_bounds__(KT) void k_kmeans_grid(const KMJob* jobs, KMJob single, int G, int k, int max_iter,
                                                    int e2, KMSlot* slots, KMSync* syncs) {
#pragma clang fp contract(off)
  __shared__ KMLocal sh;
  const int seg = blockIdx.x / G, g = blockIdx.x - seg * G;
  const KMJob J = jobs ? jobs[seg] : single;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  if (tid == 0) sh.flag = 0;
  const long long chunk = (J.n + G - 1) / G;
  const long long i0 = min(J.n, (long long)g * chunk), i1 = min(J.n, i0 + chunk);
  KMSync* sy = syncs + seg;
  KMSlot* my = slots + ((size_t)seg * G + g) * 2;
  const KMSlot* all = slots + (size_t)seg * G * 2;
  unsigned bar = 0;
  const bool do_x = J.u != nullptr;
  const float irho = 1.f / J.rho;
  const auto src = gptr(J.src);
  const auto xo = gptr(J.x);
  const auto ahat = gptr(J.a_hat);
  const auto uu = gptr(J.u);
  const auto ll = gptr(J.lam);
  const auto labels = gptr(J.labels);

  // values of this workgroup's slice (after the optional x-update)
  float v[REG ? KVPT : 1];
  float lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  if (REG) {
#pragma unroll
    for (int e = 0; e < KVPT; ++e) {
      long long i = i0 + tid + (long long)e * KT;
      float a = 0.f;
      if (i < i1) {
        a = src[i];
        if (do_x) {
          a = km_xupdate(a, uu[i], ll[i], J.rho, irho, J.eta2, e2);
          xo[i] = a;
        }
        bad |= !isfinite(a);
        lo = fminf(lo, a);
        hi = fmaxf(hi, a);
      }
      v[e] = a;
    }
  } else {
    for (long long i = i0 + tid; i < i1; i += KT) {
      float a = src[i];
      if (do_x) {
        a = km_xupdate(a, uu[i], ll[i], J.rho, irho, J.eta2, e2);
        xo[i] = a;
      }
      bad |= !isfinite(a);
      lo = fminf(lo, a);
      hi = fmaxf(hi, a);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
    bad |= __shfl_xor(bad, o, 64);
  }
  if (l == 0) { sh.red[2 * w] = lo; sh.red[2 * w + 1] = hi; sh.redb[w] = bad; }
  __syncthreads();
  if (tid == 0) {
    float a = sh.red[0], b = sh.red[1];
    int c = sh.redb[0];
    for (int i = 1; i < KWAVES; ++i) { a = fminf(a, sh.red[2 * i]); b = fmaxf(b, sh.red[2 * i + 1]); c |= sh.redb[i]; }
    if (G == 1) {
      sh.gmn[0] = a; sh.gmx[0] = b; sh.gflag[0] = c;
    } else {
      put(&my[0].mn, a);
      put(&my[0].mx, b);
      put(&my[0].bad, c);
    }
  }
  bool ok = seg_barrier(sy, G, ++bar, sh);
  if (G > 1 && tid < G) {          // every workgroup's range, loaded in parallel
    sh.gmn[tid] = get(&all[2 * tid].mn);
    sh.gmx[tid] = get(&all[2 * tid].mx);
    sh.gflag[tid] = get(&all[2 * tid].bad);
  }
  __syncthreads();
  lo = INFINITY; hi = -INFINITY; bad = 0;
  for (int q = 0; q < G; ++q) {
    lo = fminf(lo, sh.gmn[q]);
    hi = fmaxf(hi, sh.gmx[q]);
    bad |= sh.gflag[q];
  }
  if (!ok || bad || hi == lo) {
    // constant slice: one cluster at lo; non-finite input or lost barrier: flagged
    const int code = !ok ? -2 : (bad ? -1 : 0);
    for (long long i = i0 + tid; i < i1; i += KT) {
      if (J.labels) labels[i] = 0;
      if (J.a_hat && J.a_hat != J.src) ahat[i] = src[i];
    }
    if (g == 0) {
      if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = code == 0 ? lo : 0.f;
      if (J.iters && tid == 0) *J.iters = code;
    }
    seg_leave(sy, G);
    return;
  }
  int e;
  frexp(fmax(fabs((double)lo), fabs((double)hi)), &e);
  const int S = 30 - e;
  if (tid < k) {
    double lo64 = lo, hi64 = hi;
    double t = (hi64 - lo64) * (double)(2 * tid + 1);
    t = t / (double)(2 * k);
    sh.cent[tid] = (float)(lo64 + t);
  }
  __syncthreads();

  // centre order decides which (equivalent) assignment routine is used
  int steps = 0;
  while ((1 << steps) <= k) ++steps;
  auto assign = [&](float val) -> int {
    return (k > 8 && sh.sorted) ? km_assign_sorted(val, sh.cent, k, steps) : km_assign(val, sh.cent, k);
  };
  if (tid == 0) {
    int srt = 1;
    for (int j = 1; j < k; ++j) srt &= !(sh.cent[j] < sh.cent[j - 1]);
    sh.sorted = srt;
  }
  __syncthreads();

  uint8_t lab[REG ? KVPT : 1];
  if (REG) {
    assign_regs(v, lab, sh.cent, k, steps, sh.sorted);
  } else {
    for (long long i = i0 + tid; i < i1; i += KT) labels[i] = (uint8_t)assign(src[i]);
  }

  const int ncopy = k * KCOPY <= KM_MAX_K ? KCOPY : 1;
  const int nbins = k * ncopy;
  int changed = 1, it = 0;
  for (int t = 1; t <= max_iter; ++t) {
    // cluster sums of the current labels (exact integer sums: any order)
    for (int j = l; j < nbins; j += 64) { sh.sum[w][j] = 0ull; sh.cnt[w][j] = 0u; }
    __syncthreads();
    if (REG) {
#pragma unroll
      for (int q = 0; q < KVPT; ++q) {
        long long i = i0 + tid + (long long)q * KT;
        if (i < i1) {
          int bin = lab[q] * ncopy + (l & (ncopy - 1));
          atomicAdd(&sh.sum[w][bin], (unsigned long long)(long long)km_fixed(v[q], S));
          atomicAdd(&sh.cnt[w][bin], 1u);
        }
      }
    } else {
      for (long long i = i0 + tid; i < i1; i += KT) {
        int bin = labels[i] * ncopy + (l & (ncopy - 1));
        atomicAdd(&sh.sum[w][bin], (unsigned long long)(long long)km_fixed(src[i], S));
        atomicAdd(&sh.cnt[w][bin], 1u);
      }
    }
    if (changed) sh.flag = 1;
    __syncthreads();
    // this workgroup's totals: into the shared table directly (G == 1) or
    // published for the other workgroups of the segment
    KMSlot* slot = my + (t & 1);
    // fold the waves' bins into wave 0's row, then the replicas of a cluster
    for (int b = tid; b < nbins; b += KT) {
      unsigned long long q = 0;
      unsigned c = 0;
#pragma unroll
      for (int ww = 0; ww < KWAVES; ++ww) { q += sh.sum[ww][b]; c += sh.cnt[ww][b]; }
      sh.sum[0][b] = q;
      sh.cnt[0][b] = c;
    }
    __syncthreads();
    for (int j = tid; j < k; j += KT) {
      long long q = 0;
      unsigned c = 0;
      for (int r = 0; r < ncopy; ++r) { q += (long long)sh.sum[0][j * ncopy + r]; c += sh.cnt[0][j * ncopy + r]; }
      if (G == 1) {
        sh.gsum[0][j] = q;
        sh.gcnt[0][j] = c;
      } else {
        put(&slot->sum[j], q);
        put(&slot->cnt[j], c);
      }
    }
    if (tid == 0) {
      if (G == 1) sh.gflag[0] = sh.flag;
      else put(&slot->changed, sh.flag);
      sh.flag = 0;
    }
    ok = seg_barrier(sy, G, ++bar, sh);
    if (!ok) break;
    if (G > 1) {                      // all published totals, loaded in parallel
      for (int idx = tid; idx < G * k; idx += KT) {
        int gg = idx / k, j = idx - gg * k;
        sh.gsum[gg][j] = get(&all[2 * gg + (t & 1)].sum[j]);
        sh.gcnt[gg][j] = get(&all[2 * gg + (t & 1)].cnt[j]);
      }
      if (tid < G) sh.gflag[tid] = get(&all[2 * tid + (t & 1)].changed);
    }
    __syncthreads();
    // did any slice change its labels in the previous reassignment?
    int any = 0;
    for (int q = 0; q < G; ++q) any |= sh.gflag[q];
    if (t > 1 && !any) break;          // labels of iteration t-1 are final
    it = t;
    if (tid < k) {
      long long q = 0;
      unsigned long long c = 0;
      for (int gg = 0; gg < G; ++gg) { q += sh.gsum[gg][tid]; c += sh.gcnt[gg][tid]; }
      if (c > 0) sh.cent[tid] = (float)(ldexp((double)q, -S) / (double)c);
    }
    __syncthreads();
    if (tid == 0) {
      int srt = 1;
      for (int j = 1; j < k; ++j) srt &= !(sh.cent[j] < sh.cent[j - 1]);
      sh.sorted = srt;
    }
    __syncthreads();
    changed = 0;
    if (REG) {
      uint8_t nl[REG ? KVPT : 1];
      assign_regs(v, nl, sh.cent, k, steps, sh.sorted);
#pragma unroll
      for (int q = 0; q < KVPT; ++q) {
        long long i = i0 + tid + (long long)q * KT;
        if (i < i1 && nl[q] != lab[q]) changed = 1;
        lab[q] = nl[q];
      }
    } else {
      for (long long i = i0 + tid; i < i1; i += KT) {
        int nl = assign(src[i]);
        if (nl != labels[i]) { changed = 1; labels[i] = (uint8_t)nl; }
      }
    }
    __syncthreads();
  }
  if (!ok) {
    if (g == 0 && J.iters && tid == 0) *J.iters = -2;
    seg_leave(sy, G);
    return;
  }
  if (REG) {
#pragma unroll
    for (int q = 0; q < KVPT; ++q) {
      long long i = i0 + tid + (long long)q * KT;
      if (i < i1) {
        if (J.labels) labels[i] = lab[q];
        if (J.a_hat) ahat[i] = sh.cent[lab[q]];
      }
    }
  } else if (J.a_hat) {
    for (long long i = i0 + tid; i < i1; i += KT) ahat[i] = sh.cent[labels[i]];
  }
  if (g == 0) {
    if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = sh.cent[j];
    if (J.iters && tid == 0) *J.iters = it;
  }
  seg_leave(sy, G);
}

template __global__ void k_kmeans_grid<true>(const KMJob*, KMJob, int, int, int, int, KMSlot*, KMSync*);
template __global__ void k_kmeans_grid<false>(const KMJob*, KMJob, int, int, int, int, KMSlot*, KMSync*);

}  // namespace tomo
