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
// LDS rows are 16-byte aligned so whole float4s are staged with one store, and
// transposed staging assigns consecutive image rows to consecutive lanes, so
// neither staging pattern has bank conflicts.
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

template <int R, class Src>
__global__ __launch_bounds__(PTHREADS) void k_project(Src src) {
  using B = Band<R>;
  __shared__ __align__(16) float band[R * B::LS];
  __shared__ float acc[PA * PACC];
  __shared__ AngleParam prm[PA];

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
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);

  int gr0, gc0, gh, gw;
  region_of(J, region, gr0, gc0, gh, gw);

  if (tid < PA) {
    AngleParam p;
    p.cls = -1;
    p.xi0 = p.beta = p.gamma = p.rlo0 = p.rhi0 = p.rsl = 0.0;
    p.scale = 0.f;
    p.bbase = 0;
    if (tid < na) {
      double th = J.ang[a0 + tid];
      double cs = cos(th), sn = sin(th);
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
    }
    prm[tid] = p;
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

    __syncthreads();
    for (int i = tid; i < R * B::LS; i += PTHREADS) band[i] = 0.f;

    for (int db = 0; db < D; db += R) {
      __syncthreads();
      // stage R driving lines of the region (lines beyond D are zero)
      const int nl = min(R, D - db);
      if (cls == 0) {
        if (vec4) {
          const int W4 = W >> 2;
          for (int i = wave; i < R; i += NW) {
            float4* dst = reinterpret_cast<float4*>(band + i * B::LS + B::PAD);
            const float4* srow = reinterpret_cast<const float4*>(J.img + (size_t)(gr0 + db + i) * J.n + gc0);
            for (int k = lane; k < W4; k += 64) dst[k] = i < nl ? srow[k] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        } else {
          for (int i = wave; i < R; i += NW) {
            float* dst = band + i * B::LS + B::PAD;
            const float* srow = J.img + (size_t)(gr0 + db + i) * J.n + gc0;
            for (int k = lane; k < W; k += 64) dst[k] = i < nl ? srow[k] : 0.f;
          }
        }
      } else {
        // lane -> image row k, each wave stages groups of 4 band columns
        if (vec4) {
          for (int k0 = 0; k0 < W; k0 += 64) {
            const int k = k0 + lane;
            for (int q = wave; q < R / 4; q += NW) {
              const int c = db + 4 * q;
              float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
              if (k < W && c < D) v = *reinterpret_cast<const float4*>(J.img + (size_t)(gr0 + k) * J.n + gc0 + c);
              if (k < W) {
                float* dst = band + 4 * q * B::LS + B::PAD + k;
                dst[0] = v.x;                // D is a multiple of 4 here, so c < D covers c+3
                dst[B::LS] = v.y;
                dst[2 * B::LS] = v.z;
                dst[3 * B::LS] = v.w;
              }
            }
          }
        } else {
          for (int k0 = 0; k0 < W; k0 += 64) {
            const int k = k0 + lane;
            if (k >= W) continue;
            for (int i = wave; i < R; i += NW) {
              float v = i < nl ? J.img[(size_t)(gr0 + k) * J.n + gc0 + db + i] : 0.f;
              band[i * B::LS + B::PAD + k] = v;
            }
          }
        }
      }
      __syncthreads();

      // rays of each angle of this class that meet the band (wave-uniform)
      int jlo[PA], jhi[PA], nch[PA];
      int tot = 0;
#pragma unroll
      for (int a = 0; a < PA; ++a) {
        jlo[a] = 0;
        jhi[a] = -1;
        nch[a] = 0;
        if (a < na && prm[a].cls == cls) {
          const int bb = prm[a].bbase;
          int jl = max((int)floor(prm[a].rlo0 + db * prm[a].rsl), max(0, -bb));
          int jh = min((int)ceil(prm[a].rhi0 + db * prm[a].rsl), min(PACC - 1, J.nb - 1 - bb));
          jlo[a] = jl;
          jhi[a] = jh;
          nch[a] = jh >= jl ? ((jh - jl + 1 + 63) >> 6) : 0;
        }
        tot += nch[a];
      }
      // each wave takes chunks of 64 consecutive rays of one angle
      for (int ch = wave; ch < tot; ch += NW) {
        int a = 0, base = 0;
#pragma unroll
        for (int q = 0; q < PA - 1; ++q) {
          if (ch >= base + nch[a]) { base += nch[a]; ++a; }
        }
        int ja = 0, jb = -1;
#pragma unroll
        for (int q = 0; q < PA; ++q) if (q == a) { ja = jlo[q]; jb = jhi[q]; }
        const int j = ja + ((ch - base) << 6) + lane;
        if (j > jb) continue;
        const AngleParam& p = prm[a];
        const float xi = (float)(p.xi0 + db * p.gamma + (double)j * p.beta);
        const float g = (float)p.gamma;
        float s0 = 0.f, s1 = 0.f;
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
}

// Sum of the regions' partial ray sums, one thread per (angle chunk, bin):
// out = scale * sum_regions partial - d, regions added in region order.  A job
// spans n_achunk * ceil(nb / PTHREADS) workgroups of this launch.
template <class Src>
__global__ __launch_bounds__(PTHREADS) void k_project_reduce(Src src) {
  __shared__ int fin_bbase[PMAXREG * PA];
  int lid;
  const ProjJob J = src.get(blockIdx.x, lid);
  const int G = J.n_rr * J.n_rc;
  const int nbb = (J.nb + PTHREADS - 1) / PTHREADS;
  const int achunk = lid / nbb;
  const int b = (lid - achunk * nbb) * PTHREADS + threadIdx.x;
  const int a0 = achunk * PA;
  const int na = min(PA, J.n_ang - a0);
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);
  for (int i = threadIdx.x; i < G * PA; i += PTHREADS) {
    int g = i / PA, a = i - g * PA;
    int bb = 0;
    if (a < na) {
      int r0, c0, rh, rw;
      region_of(J, g, r0, c0, rh, rw);
      double th = J.ang[a0 + a];
      bb = region_bbase(cos(th), sin(th), h, hb, r0, c0, rh, rw);
    }
    fin_bbase[i] = bb;
  }
  __syncthreads();
  if (b >= J.nb) return;
  const float* pbase = J.partial + (size_t)achunk * G * (PA * PACC);
  float s[PA] = {};
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int a = 0; a < PA; ++a) {
      int j = b - fin_bbase[g * PA + a];
      if (a < na && j >= 0 && j < PACC) s[a] += pbase[((size_t)g * PA + a) * PACC + j];
    }
  }
#pragma unroll
  for (int a = 0; a < PA; ++a) {
    if (a < na) {
      size_t o = (size_t)(a0 + a) * J.nb + b;
      float v = s[a] * J.scale;
      J.out[o] = J.d ? v - J.d[o] : v;
    }
  }
}

template __global__ void k_project<16, Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project<16, Many<ProjJob>>(Many<ProjJob>);
template __global__ void k_project<32, Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project<32, Many<ProjJob>>(Many<ProjJob>);
template __global__ void k_project_reduce<Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project_reduce<Many<ProjJob>>(Many<ProjJob>);

}  // namespace tomo
