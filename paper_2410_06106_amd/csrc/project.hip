// Forward projector d = P u (Eq. 2-4) for gfx950: Joseph ray-driven
// interpolation with the image streamed through LDS in bands.
//
// A workgroup owns PA angles of one job and one rectangular image region.
// For every angle it walks the rays that cross the region along the driving
// axis (rows when |cos| >= |sin|, columns otherwise) and interpolates linearly
// between the two nearest pixels of each row (column); the region is staged in
// LDS one band of R rows (columns, transposed on the fly) at a time and every
// staged band serves all PA angles.  Zero pads of R+4 samples on both sides of
// a band row mean the inner loop needs no bounds checks; pixels outside the
// region count as zero, so the regions' partial ray sums add up exactly to the
// full projection.  When a job has several regions, a second small launch adds
// the regions' partials in region order: no atomics and no cross-workgroup
// handshakes inside a launch, results are bit-reproducible.
//
// The same kernel evaluates the chord-length model of Eq. 2 (CHORD): in each
// line a ray's segment covers |gamma| samples and is split between the two
// samples it crosses in proportion to the lengths inside them (the same two
// LDS reads, a different fraction); positions are then kept in float64 because
// those weights are steep near axis-aligned angles.
//
// LDS rows are 16-byte aligned so whole float4s are staged with one store, and
// transposed staging assigns consecutive image rows to consecutive lanes, so
// neither staging pattern has bank conflicts.  With 32-line bands (whose LDS
// use limits a CU to three workgroups) the next band is loaded into registers
// while the current one is computed; 16-line bands rely on more resident
// workgroups instead.
#include "common.h"

namespace tomo {

namespace {

template <int R>
struct Band {
  static constexpr int PAD = R + 4;                 // zero samples on each side of a band row
  static constexpr int LS = PREG + 2 * PAD;         // LDS row stride in floats (multiple of 4)
};

struct AngleParam {
  double xi0;     // interpolation coordinate of ray j = 0 at driving index 0 (LDS units)
  double beta;    // d(xi)/dj
  double gamma;   // d(xi)/d(driving index)
  double rlo0;    // first candidate ray of the band at driving index 0 (affine in it)
  double rhi0;    // last candidate ray of the band at driving index 0
  double rsl;     // slope of both with the band's first driving index
  float g32;      // gamma rounded to float32
  float scale;    // path length per step: 1/|cos| or 1/|sin|
  int cls;        // 0 row-driven, 1 column-driven, -1 inactive
  int bbase;      // detector bin of ray j = 0 for this region
};

// Lowest bin whose ray can meet a pixel of the region: floor of the smallest
// bin coordinate s = (c - h) cos + (r - h) sin + hb over the region corners.
__device__ __forceinline__ int region_bbase(double cs, double sn, double h, double hb,
                                            int gr0, int gc0, int gh, int gw) {
  double s00 = (gc0 - h) * cs + (gr0 - h) * sn + hb;
  double dc = (gw - 1) * cs, dr = (gh - 1) * sn;
  return (int)floor(s00 + fmin(0.0, dc) + fmin(0.0, dr));
}

__device__ __forceinline__ void region_of(const ProjJob& J, int region, int& gr0, int& gc0,
                                          int& gh, int& gw) {
  int rr = region / J.n_rc, rc = region - rr * J.n_rc;
  gr0 = rr * J.reg_h;
  gc0 = rc * J.reg_w;
  gh = min(J.reg_h, J.n - gr0);
  gw = min(J.reg_w, J.n - gc0);
}

}  // namespace

template <int R, class Src, bool CHORD>
__global__ __launch_bounds__(PTHREADS) void k_project(Src src) {
  using B = Band<R>;
  __shared__ __align__(16) float band[R * B::LS];
  __shared__ float acc[PA * PACC];
  __shared__ AngleParam prm[PA];
  __shared__ float inv_tau[CHORD ? PA : 1];   // chord lengths: 1 / |gamma| (1e30 when axis-aligned)

  int lid;
  const ProjJob J = src.get(blockIdx.x, lid);
  const int G = J.n_rr * J.n_rc;
  const int achunk = lid / G;
  const int region = lid - achunk * G;
  const int a0 = achunk * PA;
  const int na = min(PA, J.n_ang - a0);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int NW = PTHREADS / 64;
  static_assert(NW == 4 && PREG == 4 * 64 && R % 16 == 0, "staging assumes 4 waves and 256-wide regions");
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);

  int gr0, gc0, gh, gw;
  region_of(J, region, gr0, gc0, gh, gw);

  if (tid < PA) {
    AngleParam p;
    p.cls = -1;
    p.xi0 = p.beta = p.gamma = p.rlo0 = p.rhi0 = p.rsl = 0.0;
    p.scale = p.g32 = 0.f;
    p.bbase = 0;
    float it = 0.f;
    if (tid < na) {
      double cs, sn;
      angle_trig(J.ang[a0 + tid], CHORD, cs, sn);
      p.bbase = region_bbase(cs, sn, h, hb, gr0, gc0, gh, gw);
      double ib, W;
      if (fabs(cs) >= fabs(sn)) {   // walk rows, interpolate across columns
        p.cls = 0;
        p.beta = 1.0 / cs;
        ib = cs;
        p.gamma = -sn / cs;
        p.xi0 = (p.bbase - hb - (gr0 - h) * sn) / cs + h - gc0 + B::PAD;
        p.scale = (float)(1.0 / fabs(cs));
        W = gw;
      } else {                      // walk columns, interpolate across rows
        p.cls = 1;
        p.beta = 1.0 / sn;
        ib = sn;
        p.gamma = -cs / sn;
        p.xi0 = (p.bbase - hb - (gc0 - h) * cs) / sn + h - gr0 + B::PAD;
        p.scale = (float)(1.0 / fabs(sn));
        W = gh;
      }
      // rays j with PAD-1 < xi(j, d) < PAD+W for some driving index d of the
      // band [db, db+R): both bounds are affine in db with slope -gamma/beta
      const double span = (R - 1) * p.gamma;
      const double t1 = (B::PAD - 1 - p.xi0 - fmax(0.0, span)) * ib;
      const double t2 = (B::PAD + W - p.xi0 - fmin(0.0, span)) * ib;
      p.rlo0 = fmin(t1, t2);
      p.rhi0 = fmax(t1, t2);
      p.rsl = -p.gamma * ib;
      p.g32 = (float)p.gamma;
      if (CHORD) {
        // chord lengths: the ray's segment in a line spans |gamma| samples
        // centred on xi; it is split between the samples floor(xi + (1-|gamma|)/2)
        // and the next one, the next one taking max(0, 1 - q / |gamma|) of it,
        // q = the distance from that point to the next sample boundary
        const double tau = fabs(p.gamma);
        p.xi0 += 0.5 * (1.0 - tau);
        it = tau > 0.0 ? (float)(1.0 / tau) : 1e30f;
      }
    }
    prm[tid] = p;
    if (CHORD) inv_tau[tid] = it;
  }
  for (int i = tid; i < PA * PACC; i += PTHREADS) acc[i] = 0.f;
  __syncthreads();

  // whole-float4 staging needs 16-byte aligned rows and region corners
  const bool vec4 = ((J.n & 3) == 0) && ((gc0 & 3) == 0) && ((gw & 3) == 0) &&
                    ((reinterpret_cast<uintptr_t>(J.img) & 15) == 0);

  for (int cls = 0; cls < 2; ++cls) {
    bool any = false;
    for (int a = 0; a < na; ++a) any |= (prm[a].cls == cls);
    if (!any) continue;
    const int D = cls == 0 ? gh : gw;   // driving extent
    const int W = cls == 0 ? gw : gh;   // interpolation extent

    // R driving lines [db, db + R) of the region pass through R registers
    // per thread, loaded one band ahead of the band being computed (lines
    // beyond D and samples beyond W are zero)
    float st[R];
    auto load = [&](int db) {
      const int nl = min(R, D - db);
      if (cls == 0) {
        if (vec4) {
          const int W4 = W >> 2;
#pragma unroll
          for (int m = 0; m < R / NW; ++m) {
            const int i = wave + NW * m;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i < nl && lane < W4)
              v = reinterpret_cast<const float4*>(J.img + (size_t)(gr0 + db + i) * J.n + gc0)[lane];
            st[4 * m] = v.x; st[4 * m + 1] = v.y; st[4 * m + 2] = v.z; st[4 * m + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int m = 0; m < R / NW; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int i = wave + NW * m, k = lane + 64 * c;
              st[4 * m + c] = (i < nl && k < W) ? J.img[(size_t)(gr0 + db + i) * J.n + gc0 + k] : 0.f;
            }
        }
      } else {
        // lane -> image row k; groups of 4 consecutive band lines per float4
        if (vec4) {
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < R / 16; ++m) {
              const int k = lane + 64 * c, col = db + 4 * (wave + NW * m);
              float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
              if (k < W && col < D)   // D is a multiple of 4 here, so col < D covers col + 3
                v = *reinterpret_cast<const float4*>(J.img + (size_t)(gr0 + k) * J.n + gc0 + col);
              const int o = 4 * (c * (R / 16) + m);
              st[o] = v.x; st[o + 1] = v.y; st[o + 2] = v.z; st[o + 3] = v.w;
            }
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < R / NW; ++m) {
              const int k = lane + 64 * c, i = wave + NW * m;
              st[c * (R / NW) + m] = (k < W && i < nl) ? J.img[(size_t)(gr0 + k) * J.n + gc0 + db + i] : 0.f;
            }
        }
      }
    };
    auto store = [&]() {
      if (cls == 0) {
        if (vec4) {
#pragma unroll
          for (int m = 0; m < R / NW; ++m) {
            const int i = wave + NW * m;
            if (lane < (W >> 2))
              reinterpret_cast<float4*>(band + i * B::LS + B::PAD)[lane] =
                  make_float4(st[4 * m], st[4 * m + 1], st[4 * m + 2], st[4 * m + 3]);
          }
        } else {
#pragma unroll
          for (int m = 0; m < R / NW; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int i = wave + NW * m, k = lane + 64 * c;
              if (k < W) band[i * B::LS + B::PAD + k] = st[4 * m + c];
            }
        }
      } else {
        if (vec4) {
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < R / 16; ++m) {
              const int k = lane + 64 * c, q = wave + NW * m;
              const int o = 4 * (c * (R / 16) + m);
              if (k < W) {
                float* dst = band + 4 * q * B::LS + B::PAD + k;
                dst[0] = st[o];
                dst[B::LS] = st[o + 1];
                dst[2 * B::LS] = st[o + 2];
                dst[3 * B::LS] = st[o + 3];
              }
            }
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int m = 0; m < R / NW; ++m) {
              const int k = lane + 64 * c, i = wave + NW * m;
              if (k < W) band[i * B::LS + B::PAD + k] = st[c * (R / NW) + m];
            }
        }
      }
    };

    __syncthreads();
    for (int i = tid; i < R * B::LS; i += PTHREADS) band[i] = 0.f;
    constexpr bool prefetch = R == 32;
    if (prefetch) load(0);
    for (int db = 0; db < D; db += R) {
      __syncthreads();
      if (!prefetch) load(db);
      store();
      __syncthreads();
      if (prefetch && db + R < D) load(db + R);

      // rays of the angles of this class that meet the band, all angles in
      // one list (wave-uniform bookkeeping, kept in scalar registers)
      int base[PA], off[PA];
      int tot = 0;
#pragma unroll
      for (int a = 0; a < PA; ++a) {
        int cnt = 0, jl = 0;
        if (a < na && prm[a].cls == cls) {
          const int bb = prm[a].bbase;
          jl = max((int)floor(prm[a].rlo0 + db * prm[a].rsl), max(0, -bb));
          const int jh = min((int)ceil(prm[a].rhi0 + db * prm[a].rsl), min(PACC - 1, J.nb - 1 - bb));
          cnt = max(0, jh - jl + 1);
        }
        base[a] = __builtin_amdgcn_readfirstlane(tot);
        off[a] = __builtin_amdgcn_readfirstlane(jl - tot);
        tot = __builtin_amdgcn_readfirstlane(tot + cnt);
      }
      // each wave takes chunks of 64 consecutive entries of the list; a lane
      // finds its angle from the list offsets
      for (int q0 = wave * 64; q0 < tot; q0 += NW * 64) {
        const int q = q0 + lane;
        if (q >= tot) continue;
        int a = 0, jo = off[0];
#pragma unroll
        for (int t = 1; t < PA; ++t) {
          const bool ge = q >= base[t];
          a = ge ? t : a;
          jo = ge ? off[t] : jo;
        }
        const int j = q + jo;
        const AngleParam& p = prm[a];
        float s0 = 0.f, s1 = 0.f;
        if (CHORD) {
          // positions in float64: the weights are steep in the position near
          // axis-aligned angles (slope 1 / |gamma|)
          const double xd = p.xi0 + db * p.gamma + (double)j * p.beta;
          const float inv = inv_tau[a];
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const double xx = i == 0 ? xd : fma((double)i, p.gamma, xd);
            const int c0 = (int)xx;                           // xx > 0
            const float q = (float)((double)(c0 + 1) - xx);   // in (0, 1]
            const float f = fmaxf(0.f, fmaf(-q, inv, 1.f));
            const float v0 = band[i * B::LS + c0];
            const float v1 = band[i * B::LS + c0 + 1];
            s0 += v0;
            s1 = fmaf(f, v1 - v0, s1);
          }
        } else {
          const float xi = (float)(p.xi0 + db * p.gamma + (double)j * p.beta);
          const float g = p.g32;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            float xx = i == 0 ? xi : fmaf((float)i, g, xi);
            float f = __builtin_amdgcn_fractf(xx);   // xx > 0: truncation is the floor
            int c0 = (int)xx;
            float v0 = band[i * B::LS + c0];
            float v1 = band[i * B::LS + c0 + 1];
            s0 += v0;
            s1 = fmaf(f, v1 - v0, s1);
          }
        }
        acc[a * PACC + j] += s0 + s1;
      }
    }
  }
  __syncthreads();

  if (G == 1) {
    for (int idx = tid; idx < na * J.nb; idx += PTHREADS) {
      int a = idx / J.nb, b = idx - a * J.nb;
      int j = b - prm[a].bbase;
      float v = (j >= 0 && j < PACC) ? acc[a * PACC + j] * prm[a].scale : 0.f;
      v *= J.scale;
      size_t o = (size_t)(a0 + a) * J.nb + b;
      J.out[o] = J.d ? v - J.d[o] : v;
    }
    return;
  }

  // partial sums of this region, pre-scaled by the path length per step; a
  // separate launch (k_project_reduce) adds the regions in region order
  float* part = J.partial + ((size_t)achunk * G + region) * (PA * PACC);
  for (int i = tid; i < PA * PACC; i += PTHREADS) {
    int a = i / PACC;
    part[i] = a < na ? acc[i] * prm[a].scale : 0.f;
  }
  if (tid < PA) J.bbase[((size_t)achunk * G + region) * PA + tid] = prm[tid].bbase;
}

// Sum of the regions' partial ray sums, one thread per (angle chunk, bin):
// out = scale * sum_regions partial - d, regions added in region order.  A job
// spans n_achunk * ceil(nb / PTHREADS) workgroups of this launch.
template <class Src>
__global__ __launch_bounds__(PTHREADS) void k_project_reduce(Src src) {
  int lid;
  const ProjJob J = src.get(blockIdx.x, lid);
  const int G = J.n_rr * J.n_rc;
  const int nbb = (J.nb + PTHREADS - 1) / PTHREADS;
  const int achunk = lid / nbb;
  const int b = (lid - achunk * nbb) * PTHREADS + threadIdx.x;
  const int a0 = achunk * PA;
  const int na = min(PA, J.n_ang - a0);
  // first bins of the regions' partials, as the projector computed them: the
  // same for every thread of the workgroup, so read through the constant
  // address space (scalar loads, no LDS staging or barrier)
  const auto fin_bbase = (const __attribute__((address_space(4))) int*)(J.bbase + (size_t)achunk * G * PA);
  if (b >= J.nb) return;
  const float* pbase = J.partial + (size_t)achunk * G * (PA * PACC);
  // every region wrote all PA * PACC of its partials (zeros past its rays), so
  // the loads are clamped into range and issued unconditionally, all of a
  // region at once; the range test only selects what is added
  float s[PA] = {};
  for (int g = 0; g < G; ++g) {
    float v[PA];
    bool ok[PA];
#pragma unroll
    for (int a = 0; a < PA; ++a) {
      const int j = b - fin_bbase[g * PA + a];
      ok[a] = j >= 0 && j < PACC;
      v[a] = pbase[((size_t)g * PA + a) * PACC + min(max(j, 0), PACC - 1)];
    }
#pragma unroll
    for (int a = 0; a < PA; ++a)
      if (ok[a]) s[a] += v[a];
  }
  float dv[PA] = {};
  if (J.d) {
#pragma unroll
    for (int a = 0; a < PA; ++a) dv[a] = J.d[(size_t)(a0 + min(a, na - 1)) * J.nb + b];
  }
#pragma unroll
  for (int a = 0; a < PA; ++a) {
    if (a < na) {
      const float v = s[a] * J.scale;
      J.out[(size_t)(a0 + a) * J.nb + b] = J.d ? v - dv[a] : v;
    }
  }
}

template __global__ void k_project<16, Single<ProjJob>, false>(Single<ProjJob>);
template __global__ void k_project<16, Many<ProjJob>, false>(Many<ProjJob>);
template __global__ void k_project<32, Single<ProjJob>, false>(Single<ProjJob>);
template __global__ void k_project<32, Many<ProjJob>, false>(Many<ProjJob>);
template __global__ void k_project<16, Single<ProjJob>, true>(Single<ProjJob>);
template __global__ void k_project<16, Many<ProjJob>, true>(Many<ProjJob>);
template __global__ void k_project<32, Single<ProjJob>, true>(Single<ProjJob>);
template __global__ void k_project<32, Many<ProjJob>, true>(Many<ProjJob>);
template __global__ void k_project_reduce<Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project_reduce<Many<ProjJob>>(Many<ProjJob>);

}  // namespace tomo
