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
// For a float32 value a, 2a <= m holds exactly when a <= x(m), the largest
// float32 whose double does not exceed m / 2, so every comparison with a
// midpoint is one float32 comparison with its threshold x(m).  Because the
// label is monotone in the value, every cluster is a run of the sorted values,
// and the labelling is fixed by k - 1 boundary counts (values at or below each
// threshold).  One workgroup owns a segment.  It buckets the values once by
// value range (a monotone bucket function), keeping exclusive prefix counts and
// exact int64 prefix sums of the codes per bucket, and regroups the values by
// bucket (in LDS, or in a global workspace for long segments).  The count and
// code sum at or below a threshold are then the prefix of the buckets left of
// the threshold's bucket plus that one bucket's share: a Lloyd iteration costs
// k - 1 bucket scans instead of a pass over every value, and "no label
// changed" is "no boundary count changed".  For k <= 64 the Lloyd iterations
// run in one wave with no barrier: a group of lanes per threshold scans its
// bucket, and neighbouring groups exchange totals and centres through DPP
// shifts and lane swaps (lloyd_wave); larger k use every wave and a barrier per
// step.  Segments of up to 16384 values stay in registers from the first pass
// to the last, where labels and quantized values are written.  The optional
// Alg. 3 x-update of the segment (its closed form) is applied on load.
#include "consensus.h"

namespace tomo {

namespace {

constexpr int KT = 1024;                // threads per workgroup
constexpr int KWAVES = KT / 64;
constexpr int KVPT = 16;                // values per thread and pass (loads in flight)
constexpr int KBUCKETS = 4096;          // value-range buckets at most
constexpr int KPER = KBUCKETS / KT;     // bucket entries per thread in the scan
static_assert(KT * KVPT == KM_LDS_VALUES, "register-resident segments are the LDS-resident ones");

struct KMShared {
  int start[KBUCKETS + 1];        // bucket counts, then their exclusive prefix (start[B] = n)
  int fill[KBUCKETS];             // values placed per bucket so far
  long long psum[KBUCKETS + 1];   // code sums per bucket, then their exclusive prefix
  float thr[KM_MAX_K];            // thresholds x(c_j + c_{j+1}), increasing
  float cent[KM_MAX_K];           // centres, increasing
  float upd[KM_MAX_K];            // updated centres before sorting
  int cb[2][KM_MAX_K + 1];        // values at or below threshold j-1 (label < j), two generations
  long long sb[KM_MAX_K + 1];     // their code sums
  long long wsum[KWAVES];
  int wcnt[KWAVES];
  float red[2 * KWAVES];
  int redb[KWAVES];
};

__device__ __forceinline__ int km_fixed(float v, int S) {
  return (int)rintf(ldexpf(v, S));     // exact scaling, round half to even
}

// Alg. 3 on one value (closed form, coefficient q; E2 = 0 leaves it as it is)
__device__ __forceinline__ float km_xupdate(float xv, float uv, float lv, float irho, float q, int e2) {
  return e2 > 0 ? xseg(xv, reg_target(uv, lv, irho), q) : xv;
}

// the same with a regularization block's target t_z and penalty rho_z
__device__ __forceinline__ float km_xupdate_reg(float xv, float tm, float tv, float rho, float rho_z, float c,
                                                int e2) {
  return e2 > 0 ? xseg_reg(xv, tm, tv, rho, rho_z, c) : xv;
}

// Largest float32 below a finite x.
__device__ __forceinline__ float prev_float(float x) {
  if (x == 0.f) return __uint_as_float(0x80000001u);
  const unsigned u = __float_as_uint(x);
  return __uint_as_float(x > 0.f ? u - 1u : u + 1u);
}

// x(m): the largest float32 whose double is <= m / 2 (m / 2 is exact), so that
// a <= x(m) exactly when 2a <= m for every float32 a.  Midpoints lie between
// the smallest and largest value, so x(m) is finite.
__device__ __forceinline__ float threshold(double m) {
  const double h = 0.5 * m;
  float x = (float)h;
  if ((double)x > h) x = prev_float(x);
  return x;
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

// Cross-lane moves by DPP (every lane of the wave active): lane l reads the
// value of another lane of the wave, 0 where the pattern has no source lane.
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) { return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false); }
template <int CTRL>
__device__ __forceinline__ long long dpp_mov(long long v) {
  const unsigned lo = (unsigned)dpp_mov<CTRL>((int)v), hi = (unsigned)dpp_mov<CTRL>((int)(v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) { return __int_as_float(dpp_mov<CTRL>(__float_as_int(v))); }
__device__ __forceinline__ long long lane_value(long long v, int i) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, i);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), i);
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int lane_value(int v, int i) { return __builtin_amdgcn_readlane(v, i); }

// Inclusive prefix sum over the 64 lanes of a wave (every lane active):
// shifted adds within rows of 16 lanes (row_shr 1, 2, 4, 8), then each row
// adds the totals of the rows below it (their last lanes, read as scalars).
// Integer adds, so exact in any order.
template <typename T>
__device__ __forceinline__ T wave_scan(T v) {
  v += dpp_mov<0x111>(v);   // row_shr:1
  v += dpp_mov<0x112>(v);   // row_shr:2
  v += dpp_mov<0x114>(v);   // row_shr:4
  v += dpp_mov<0x118>(v);   // row_shr:8
  const T r0 = lane_value(v, 15), r1 = lane_value(v, 31), r2 = lane_value(v, 47);
  const int l = threadIdx.x & 63;
  if (l >= 16) v += r0;
  if (l >= 32) v += r1;
  if (l >= 48) v += r2;
  return v;
}

// Min, max and OR over the 64 lanes of a wave, to every lane: rotations within
// rows of 16 lanes, then the row pairs and the wave halves (v_permlane16_swap,
// v_permlane32_swap: the lane's own value and its partner's).
__device__ __forceinline__ float swap16(float v, bool mx) {
  const auto p = __builtin_amdgcn_permlane16_swap((unsigned)__float_as_int(v), (unsigned)__float_as_int(v), false, false);
  const float a = __int_as_float((int)p[0]), b = __int_as_float((int)p[1]);
  return mx ? fmaxf(a, b) : fminf(a, b);
}
__device__ __forceinline__ float swap32(float v, bool mx) {
  const auto p = __builtin_amdgcn_permlane32_swap((unsigned)__float_as_int(v), (unsigned)__float_as_int(v), false, false);
  const float a = __int_as_float((int)p[0]), b = __int_as_float((int)p[1]);
  return mx ? fmaxf(a, b) : fminf(a, b);
}
__device__ __forceinline__ void wave_range(float& lo, float& hi, int& bad) {
  lo = fminf(lo, dpp_mov<0x121>(lo)); hi = fmaxf(hi, dpp_mov<0x121>(hi)); bad |= dpp_mov<0x121>(bad);   // row_ror:1
  lo = fminf(lo, dpp_mov<0x122>(lo)); hi = fmaxf(hi, dpp_mov<0x122>(hi)); bad |= dpp_mov<0x122>(bad);   // row_ror:2
  lo = fminf(lo, dpp_mov<0x124>(lo)); hi = fmaxf(hi, dpp_mov<0x124>(hi)); bad |= dpp_mov<0x124>(bad);   // row_ror:4
  lo = fminf(lo, dpp_mov<0x128>(lo)); hi = fmaxf(hi, dpp_mov<0x128>(hi)); bad |= dpp_mov<0x128>(bad);   // row_ror:8
  lo = swap16(lo, false); hi = swap16(hi, true);
  lo = swap32(lo, false); hi = swap32(hi, true);
  const auto b16 = __builtin_amdgcn_permlane16_swap((unsigned)bad, (unsigned)bad, false, false);
  bad = (int)(b16[0] | b16[1]);
  const auto b32 = __builtin_amdgcn_permlane32_swap((unsigned)bad, (unsigned)bad, false, false);
  bad = (int)(b32[0] | b32[1]);
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
  const int ic = wave_scan(ct);
  const long long is = wave_scan(st);
  if (l == 63) { sh.wcnt[w] = ic; sh.wsum[w] = is; }
  __syncthreads();
  int ec = ic - ct;
  long long es = is - st;
  // the totals of the waves below: all of them read at once, those at or
  // above this wave masked (integer adds, exact in any order)
#pragma unroll
  for (int q = 0; q < KWAVES; ++q) {
    const int cq = sh.wcnt[q];
    const long long sq = sh.wsum[q];
    ec += q < w ? cq : 0;
    es += q < w ? sq : 0;
  }
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

// Sum of a 64-bit integer over the 64 lanes of a wave (every lane active),
// returned to every lane: butterflies within each row of 16 lanes (DPP quad
// permutations and the half-row and row mirrors), then the four row sums.
// Integer adds, so exact in any order.
template <int CTRL>
__device__ __forceinline__ long long dpp_add_i64(long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
  return v + (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ long long wave_sum_i64(long long v) {
  v = dpp_add_i64<0xB1>(v);    // quad_perm [1, 0, 3, 2]: pairs
  v = dpp_add_i64<0x4E>(v);    // quad_perm [2, 3, 0, 1]: quads
  v = dpp_add_i64<0x141>(v);   // row_half_mirror: lanes i and 7 - i of each half-row
  v = dpp_add_i64<0x140>(v);   // row_mirror: lanes i and 15 - i of each row
  auto lane = [&](int i) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, i);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), i);
    return (long long)(((unsigned long long)hi << 32) | lo);
  };
  return lane(0) + lane(16) + lane(32) + lane(48);
}

// Cross-lane moves of the Lloyd loop (every lane of the wave active).  Lane
// l of the wave holds group l % KP (KP a power of two): the previous group's
// lane is l - 1 and the next group's l + 1, one DPP wave shift away; the
// lanes of one group are KP apart, and their sum reaches every one of them by
// rotations within rows of 16 lanes (distances below 16), then the swaps of
// row pairs and of wave halves (v_permlane16_swap / v_permlane32_swap, whose
// two results add up to the lane's own value plus its partner's).  Integer
// adds, so exact in any order.
__device__ __forceinline__ int from_prev(int v) { return dpp_mov<0x138>(v); }        // wave_shr:1
__device__ __forceinline__ long long from_prev(long long v) { return dpp_mov<0x138>(v); }
__device__ __forceinline__ float from_next(float v) { return __int_as_float(dpp_mov<0x130>(__float_as_int(v))); }   // wave_shl:1

__device__ __forceinline__ int pair_sum16(int v) {
  const auto p = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return (int)(p[0] + p[1]);
}
__device__ __forceinline__ int pair_sum32(int v) {
  const auto p = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return (int)(p[0] + p[1]);
}
__device__ __forceinline__ long long pair_sum16(long long v) {
  const auto a = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
  return (long long)((((unsigned long long)b[0] << 32) | a[0]) + (((unsigned long long)b[1] << 32) | a[1]));
}
__device__ __forceinline__ long long pair_sum32(long long v) {
  const auto a = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
  return (long long)((((unsigned long long)b[0] << 32) | a[0]) + (((unsigned long long)b[1] << 32) | a[1]));
}
template <int KP, typename T>
__device__ __forceinline__ T strided_sum(T v) {
  if constexpr (KP <= 1) v += dpp_mov<0x121>(v);   // row_ror:1
  if constexpr (KP <= 2) v += dpp_mov<0x122>(v);   // row_ror:2
  if constexpr (KP <= 4) v += dpp_mov<0x124>(v);   // row_ror:4
  if constexpr (KP <= 8) v += dpp_mov<0x128>(v);   // row_ror:8
  if constexpr (KP <= 16) v = pair_sum16(v);
  if constexpr (KP <= 32) v = pair_sum32(v);
  return v;
}

// Count and code sum of the values a <= x for the threshold x of a group (its
// 64 / KP lanes hold the same x; `sub` is the lane's index in the group): the
// buckets left of x's bucket from the prefix tables, plus the values of that
// bucket at or below x, which the group's lanes read 64 / KP apart (four reads
// in flight per trip).  Every lane of the group gets the totals.
template <int KP, class VP>
__device__ __forceinline__ void group_at_or_below(const KMShared& sh, VP V, float x, const Buckets& bk, float lo,
                                                  float hi, int n, long long tot, int S, int sub, int& cnt,
                                                  long long& sum) {
  constexpr int G = 64 / KP;
  int c0 = 0, p0 = 0, p1 = 0;
  long long s0 = 0;
  if (x >= hi) {
    c0 = n;
    s0 = tot;
  } else if (x >= lo) {
    const int b = bk.of(x);
    p0 = sh.start[b];
    p1 = sh.start[b + 1];
    c0 = p0;
    s0 = sh.psum[b];
  }
  int c = 0;
  long long s = 0;
  for (int p = p0 + sub; p < p1; p += 4 * G) {   // four reads per trip, all in flight
    float a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = V[min(p + r * G, p1 - 1)];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (p + r * G < p1 && a[r] <= x) {
        ++c;
        s += km_fixed(a[r], S);
      }
  }
  cnt = c0 + strided_sum<KP>(c);
  sum = s0 + strided_sum<KP>(s);
}

// Lloyd iterations for k <= KP <= 64 in one wave (wave 0 of the workgroup),
// with no barrier inside the loop.  Group j (lanes j, j + KP, ...) holds
// centre j and, for j < k - 1, the threshold between centres j and j + 1,
// whose count and code sum at or below it the group's lanes find together.
// Cluster j is the values between thresholds j - 1 and j: its totals take the
// previous group's from the lane one below.  Groups from k - 1 up hold no
// threshold (+inf: all n values, the total code sum).  Every cross-lane
// operation runs with all 64 lanes active.  Returns the iterations run; the
// final centres and thresholds go to sh.cent and sh.thr.
template <int KP, class VP>
__device__ int lloyd_wave(KMShared& sh, VP V, const Buckets& bk, float lo, float hi, int n, long long tot, int S,
                          int k, int max_iter) {
  const int l = threadIdx.x & 63;
  const int grp = l & (KP - 1), sub = l / KP;
  const bool has_c = grp < k, has_t = grp < k - 1;
  float cj = has_c ? sh.cent[grp] : 0.f;
  const float c1 = from_next(cj);
  float xt = has_t ? threshold((double)cj + (double)c1) : INFINITY;
  int prev = 0, it = 0;
  for (int t = 0;; ++t) {
    int cb;
    long long sb;
    group_at_or_below<KP>(sh, V, xt, bk, lo, hi, n, tot, S, sub, cb, sb);
    if (t > 0) {
      it = t;
      if (__ballot(has_t && cb != prev) == 0) break;   // no label changed
    }
    if (t == max_iter) break;
    prev = cb;
    // centres of the current labels, then their stable sort: when they are
    // already non-decreasing the sort is the identity; otherwise every group
    // finds its stable rank (the groups' first lanes broadcast one at a time)
    // and picks the centre ranked grp
    const int cprev = from_prev(cb);
    const long long sprev = from_prev(sb);
    const int c = has_c ? cb - (grp > 0 ? cprev : 0) : 0;
    const long long q = sb - (grp > 0 ? sprev : 0);
    float u = cj;
    if (c > 0) u = (float)(ldexp((double)q, -S) / (double)c);
    float un = from_next(u);
    if (__ballot(grp + 1 < k && un < u) == 0) {
      cj = u;
    } else {
      int r = 0;
      for (int i = 0; i < k; ++i) {
        const float ui = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), i));
        r += (ui < u) || (ui == u && i < grp);
      }
      for (int i = 0; i < k; ++i) {
        const float ui = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u), i));
        cj = __builtin_amdgcn_readlane(r, i) == grp ? ui : cj;
      }
      un = from_next(cj);
    }
    xt = has_t ? threshold((double)cj + (double)un) : INFINITY;
  }
  if (sub == 0) {
    if (has_c) sh.cent[grp] = cj;
    if (has_t) sh.thr[grp] = xt;
  }
  return it;
}

// Count and code sum of the values a <= x, by one wave (every lane active and
// every lane gets the result): the buckets left of x's bucket plus the
// qualifying values of that bucket, counted with ballots and summed across
// the wave in registers.
template <class VP>
__device__ __forceinline__ void at_or_below(const KMShared& sh, VP V, float x, const Buckets& bk, float lo,
                                            float hi, int n, long long tot, int S, int& cnt, long long& sum) {
  if (x < lo) { cnt = 0; sum = 0; return; }
  if (x >= hi) { cnt = n; sum = tot; return; }
  const int b = bk.of(x);
  const int p0 = sh.start[b], p1 = sh.start[b + 1];
  const long long below = sh.psum[b];        // code sum of the buckets left of b
  const int l = threadIdx.x & 63;
  int c = 0;
  long long s = 0;
  for (int pw = p0; pw < p1; pw += 64) {     // uniform trip count: every lane sees every ballot
    const int p = pw + l;
    const float a = V[min(p, p1 - 1)];       // in the bucket (p1 > p0 here); lanes past it are masked below
    const bool in = p < p1 && a <= x;
    c += __popcll(__ballot(in));
    if (in) s += km_fixed(a, S);
  }
  cnt = p0 + c;
  sum = below + wave_sum_i64(s);
}

}  // namespace

// One workgroup per segment.  REG: the segment fits the registers (n <=
// KM_LDS_VALUES) and its bucket-ordered copy fits LDS; otherwise the values
// are streamed in every pass and the copy goes to the job's workspace.  TZ:
// jobs may carry a regularization block's target (a separate instantiation,
// so that the kernel without blocks keeps its register allocation).
template <bool REG, bool TZ>
__global__ __launch_bounds__(KT) void k_kmeans(const KMJob* jobs, KMJob single, int k, int max_iter, int e2,
                                               const KMBlock* blocks) {
#pragma clang fp contract(off)
  __shared__ KMShared sh;
  __shared__ float vlds[REG ? KM_LDS_VALUES : 1];
  const int seg = blockIdx.x;
  const KMJob J = jobs ? jobs[seg] : single;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int n = (int)J.n;
  const bool do_x = J.u != nullptr;
  const float irho = 1.f / J.rho;
  const float xq = do_x ? xseg_q(J.rho, J.eta2, e2) : 0.f;
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
  // the bucket tables are cleared first, while the first pass's loads are in
  // flight (the barrier after the range reduction orders them before use)
  const int B = min(KBUCKETS, max(1, n / 4));
  for (int b = tid; b < B; b += KT) { sh.start[b] = 0; sh.fill[b] = 0; sh.psum[b] = 0; }

  // every value once, KVPT per thread at a time: from registers (REG) or
  // loaded from the segment after the x-update
  float v[REG ? KVPT : 1];
  auto each = [&](auto&& body) {
    if constexpr (REG) {
#pragma unroll
      for (int e = 0; e < KVPT; ++e) {
        const int i = tid + e * KT;
        if (i < n) body(i, v[e]);
      }
    } else {
      for (long long base = 0; base < n; base += (long long)KT * KVPT) {
        float a[KVPT];
#pragma unroll
        for (int e = 0; e < KVPT; ++e) {   // clamped, unconditional loads: all in flight at once
          const long long i = base + tid + (long long)e * KT;
          a[e] = vals[i < n ? i : n - 1];
        }
#pragma unroll
        for (int e = 0; e < KVPT; ++e) {
          const long long i = base + tid + (long long)e * KT;
          if (i < n) body((int)i, a[e]);
        }
      }
    }
  };

  // pass 1: x-update, range, finiteness (all loads of a chunk issued first)
  float lo = INFINITY, hi = -INFINITY;
  int bad = 0;
  for (long long base = 0; base < n; base += (long long)KT * KVPT) {
    // clamped, unconditional loads (all in flight at once); a clamped slot
    // repeats the last value, which leaves the range and the flag unchanged
    float a[KVPT];
#pragma unroll
    for (int e = 0; e < KVPT; ++e) {
      const long long i = base + tid + (long long)e * KT;
      a[e] = src[i < n ? i : n - 1];
    }
    if (do_x) {
      float uv[KVPT], lv[KVPT];
#pragma unroll
      for (int e = 0; e < KVPT; ++e) {
        const long long i = base + tid + (long long)e * KT;
        uv[e] = uu[i < n ? i : n - 1];
        lv[e] = ll[i < n ? i : n - 1];
      }
      const KMBlock RB = (TZ && blocks) ? blocks[seg] : KMBlock{nullptr, 0.f};
      if (TZ && RB.tz) {
        const auto tzz = gptr(RB.tz);
        const float xc = xseg_c(J.rho, RB.rho_z, J.eta2, e2);
        // t_m = u + lambda/rho into the u registers, then t_z into the lambda
        // registers (no more values in flight than without the block)
#pragma unroll
        for (int e = 0; e < KVPT; ++e) {
          const long long i = base + tid + (long long)e * KT;
          uv[e] = reg_target(uv[e], lv[e], irho);
          lv[e] = tzz[i < n ? i : n - 1];
        }
#pragma unroll
        for (int e = 0; e < KVPT; ++e) {
          const long long i = base + tid + (long long)e * KT;
          a[e] = km_xupdate_reg(a[e], uv[e], lv[e], J.rho, RB.rho_z, xc, e2);
          if (!REG && i < n) xo[i] = a[e];   // re-read by the later passes
        }
      } else {
#pragma unroll
        for (int e = 0; e < KVPT; ++e) {
          const long long i = base + tid + (long long)e * KT;
          a[e] = km_xupdate(a[e], uv[e], lv[e], irho, xq, e2);
          if (!REG && i < n) xo[i] = a[e];   // re-read by the later passes
        }
      }
    }
    if (J.xt) {
#pragma unroll
      for (int e = 0; e < KVPT; ++e) {
        const long long i = base + tid + (long long)e * KT;
        if (i < n) gptr(J.xt)[i] = a[e];
      }
    }
#pragma unroll
    for (int e = 0; e < KVPT; ++e) {
      bad |= !isfinite(a[e]);
      lo = fminf(lo, a[e]);
      hi = fmaxf(hi, a[e]);
      if constexpr (REG) v[e] = a[e];
    }
    if constexpr (REG) break;   // n <= KT * KVPT: one chunk
  }
  wave_range(lo, hi, bad);
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
    // constant segment: one cluster at lo; non-finite input: flagged (values
    // held in registers are always written: x~ was not stored in pass 1)
    const bool copy = J.a_hat && (REG || J.a_hat != (do_x ? J.x : J.src));
    each([&](int i, float a) {
      if (J.labels) labels[i] = 0;
      if (copy) ahat[i] = a;
    });
    if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = bad ? 0.f : lo;
    if (J.iters && tid == 0) *J.iters = bad ? -1 : 0;
    return;
  }
  int e;
  frexp(fmax(fabs((double)lo), fabs((double)hi)), &e);
  const int S = 30 - e;
  const Buckets bk{lo, (float)B / (hi - lo), (float)(B - 1)};

  // pass 2: bucket counts and code sums
  if (tid < k) {
    double lo64 = lo, hi64 = hi;
    double t = (hi64 - lo64) * (double)(2 * tid + 1);
    t = t / (double)(2 * k);
    sh.cent[tid] = (float)(lo64 + t);
  }
  __syncthreads();
  each([&](int, float a) {
    const int b = bk.of(a);
    atomicAdd(&sh.start[b], 1);
    atomicAdd((unsigned long long*)&sh.psum[b], (unsigned long long)(long long)km_fixed(a, S));
  });
  __syncthreads();
  bucket_scan(sh, B);
  const long long tot = sh.psum[B];

  // pass 3: values regrouped by bucket
  float* const wv = REG ? nullptr : J.work;
  each([&](int, float a) {
    const int b = bk.of(a);
    const int p = sh.start[b] + atomicAdd(&sh.fill[b], 1);
    if constexpr (REG) vlds[p] = a;
    else gptr(wv)[p] = a;
  });
  if (tid < k - 1) sh.thr[tid] = threshold((double)sh.cent[tid] + (double)sh.cent[tid + 1]);
  if (tid == 0) {
    sh.cb[0][0] = sh.cb[1][0] = 0;
    sh.cb[0][k] = sh.cb[1][k] = n;
    sh.sb[0] = 0;
    sh.sb[k] = tot;
  }
  __syncthreads();

  auto scan_bucket = [&](float x, int& c, long long& s) {
    if constexpr (REG) at_or_below(sh, vlds, x, bk, lo, hi, n, tot, S, c, s);
    else at_or_below(sh, gptr((const float*)wv), x, bk, lo, hi, n, tot, S, c, s);
  };

  int it = 0;
  if (k <= 64) {
    // Lloyd iterations in wave 0 alone (lloyd_wave), groups of 64 / KP lanes
    if (w == 0) {
      auto run = [&](auto V) {
        if (k <= 1) return lloyd_wave<1>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
        if (k <= 2) return lloyd_wave<2>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
        if (k <= 4) return lloyd_wave<4>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
        if (k <= 8) return lloyd_wave<8>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
        if (k <= 16) return lloyd_wave<16>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
        if (k <= 32) return lloyd_wave<32>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
        return lloyd_wave<64>(sh, V, bk, lo, hi, n, tot, S, k, max_iter);
      };
      if constexpr (REG) it = run(static_cast<const float*>(vlds));
      else it = run(gptr((const float*)wv));
    }
    __syncthreads();
  } else {
    auto boundaries = [&](int gen) {
      for (int j = w; j < k - 1; j += KWAVES) {
        int c;
        long long s;
        scan_bucket(sh.thr[j], c, s);
        if (l == 0) { sh.cb[gen][j + 1] = c; sh.sb[j + 1] = s; }
      }
    };
    boundaries(0);
    __syncthreads();
    int cur = 0;
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
      if (tid < k - 1) sh.thr[tid] = threshold((double)sh.cent[tid] + (double)sh.cent[tid + 1]);
      __syncthreads();
      boundaries(cur ^ 1);
      __syncthreads();
      it = t;
      const int moved = tid <= k && sh.cb[cur ^ 1][tid] != sh.cb[cur][tid];
      cur ^= 1;
      if (!__syncthreads_or(moved)) break;
    }
  }

  // labels and quantized values: the number of thresholds below the value
  if (k <= 16) {
    float th[15];
#pragma unroll
    for (int j = 0; j < 15; ++j) th[j] = j < k - 1 ? sh.thr[j] : INFINITY;
    auto label = [&](float a) {
      int p = 0;
      if (k <= 8) {
#pragma unroll
        for (int j = 0; j < 7; ++j) p += th[j] < a ? 1 : 0;
      } else {
#pragma unroll
        for (int j = 0; j < 15; ++j) p += th[j] < a ? 1 : 0;
      }
      return p;
    };
    each([&](int i, float a) {
      const int p = label(a);
      if (J.labels) labels[i] = (uint8_t)p;
      if (J.a_hat) ahat[i] = sh.cent[p];
    });
  } else {
    each([&](int i, float a) {
      int p = 0, len = k - 1;
      while (len > 0) {
        const int half = len >> 1;
        if (sh.thr[p + half] < a) { p += half + 1; len -= half + 1; }
        else len = half;
      }
      if (J.labels) labels[i] = (uint8_t)p;
      if (J.a_hat) ahat[i] = sh.cent[p];
    });
  }
  if (J.cent) for (int j = tid; j < k; j += KT) J.cent[j] = sh.cent[j];
  if (J.iters && tid == 0) *J.iters = it;
}

template __global__ void k_kmeans<true, false>(const KMJob*, KMJob, int, int, int, const KMBlock*);
template __global__ void k_kmeans<false, false>(const KMJob*, KMJob, int, int, int, const KMBlock*);
template __global__ void k_kmeans<true, true>(const KMJob*, KMJob, int, int, int, const KMBlock*);
template __global__ void k_kmeans<false, true>(const KMJob*, KMJob, int, int, int, const KMBlock*);

}  // namespace tomo
