// Forward projector d = P u (Eq. 2-4) for gfx950: Joseph ray-driven
// interpolation with the image streamed through LDS in bands.
//
// A workgroup owns PA angles of one job and one rectangular image region.
// For every angle it walks the rays that cross the region along the driving
// axis (rows when |cos| >= |sin|, columns otherwise) and interpolates linearly
// between the two nearest pixels of each row (column); the region is staged in
// LDS one band of R rows (columns, transposed on the fly) at a time and every
// staged band serves all PA angles.  LDS pads of R+3 zero samples on both sides
// of a band row mean the inner loop needs no bounds checks; pixels outside the
// region count as zero, so the region's partial ray sums add up exactly to the
// full projection.  The last workgroup of an angle chunk (ticket counter) adds
// the partials of all regions in region order: no atomics on data, results are
// bit-reproducible.
#include "common.h"

namespace tomo {

namespace {

constexpr int PR = 16;                         // band depth (driving direction)
constexpr int PPAD = PR + 3;                   // zero pad on each side of a band row
constexpr int PLS = PREG + 2 * PPAD + 1;       // LDS row stride in floats (odd)

struct AngleParam {
  double xi0;     // interpolation coordinate of ray j = 0 at driving index 0 (LDS units)
  double beta;    // d(xi)/dj
  double gamma;   // d(xi)/d(driving index)
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

template <class Src>
__global__ __launch_bounds__(PTHREADS) void k_project(Src src) {
  __shared__ float band[PR * PLS];
  __shared__ float acc[PA * PACC];
  __shared__ AngleParam prm[PA];
  __shared__ int s_last;
  __shared__ int fin_bbase[64 * PA];

  int lid;
  const ProjJob J = src.get(blockIdx.x, lid);
  const int G = J.n_rr * J.n_rc;
  const int achunk = lid / G;
  const int region = lid - achunk * G;
  const int a0 = achunk * PA;
  const int na = min(PA, J.n_ang - a0);
  const int tid = threadIdx.x;
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);

  int gr0, gc0, gh, gw;
  region_of(J, region, gr0, gc0, gh, gw);

  if (tid < PA) {
    AngleParam p;
    p.cls = -1;
    p.xi0 = p.beta = p.gamma = 0.0;
    p.scale = 0.f;
    p.bbase = 0;
    if (tid < na) {
      double th = J.ang[a0 + tid];
      double cs = cos(th), sn = sin(th);
      p.bbase = region_bbase(cs, sn, h, hb, gr0, gc0, gh, gw);
      if (fabs(cs) >= fabs(sn)) {   // walk rows, interpolate across columns
        p.cls = 0;
        p.beta = 1.0 / cs;
        p.gamma = -sn / cs;
        p.xi0 = (p.bbase - hb - (gr0 - h) * sn) / cs + h - gc0 + PPAD;
        p.scale = (float)(1.0 / fabs(cs));
      } else {                      // walk columns, interpolate across rows
        p.cls = 1;
        p.beta = 1.0 / sn;
        p.gamma = -cs / sn;
        p.xi0 = (p.bbase - hb - (gc0 - h) * cs) / sn + h - gr0 + PPAD;
        p.scale = (float)(1.0 / fabs(sn));
      }
    }
    prm[tid] = p;
  }
  for (int i = tid; i < PA * PACC; i += PTHREADS) acc[i] = 0.f;
  __syncthreads();

  for (int cls = 0; cls < 2; ++cls) {
    bool any = false;
    for (int a = 0; a < na; ++a) any |= (prm[a].cls == cls);
    if (!any) continue;
    const int D = cls == 0 ? gh : gw;   // driving extent
    const int W = cls == 0 ? gw : gh;   // interpolation extent

    __syncthreads();
    for (int i = tid; i < PR * PLS; i += PTHREADS) band[i] = 0.f;

    for (int db = 0; db < D; db += PR) {
      __syncthreads();
      // stage R driving lines of the region (zero beyond D)
      if (cls == 0) {
        for (int idx = tid; idx < PR * W; idx += PTHREADS) {
          int i = idx / W, k = idx - i * W;
          float v = 0.f;
          if (db + i < D) v = J.img[(size_t)(gr0 + db + i) * J.n + gc0 + k];
          band[i * PLS + PPAD + k] = v;
        }
      } else {
        for (int idx = tid; idx < PR * W; idx += PTHREADS) {
          int k = idx / PR, i = idx - k * PR;
          float v = 0.f;
          if (db + i < D) v = J.img[(size_t)(gr0 + k) * J.n + gc0 + db + i];
          band[i * PLS + PPAD + k] = v;
        }
      }
      __syncthreads();

      // rays of each angle of this class that meet the band
      int jlo[PA], cnt[PA], pre[PA + 1];
      pre[0] = 0;
#pragma unroll
      for (int a = 0; a < PA; ++a) {
        jlo[a] = 0;
        cnt[a] = 0;
        if (a < na && prm[a].cls == cls) {
          const AngleParam p = prm[a];
          double e0 = p.xi0 + db * p.gamma, e1 = p.xi0 + (db + PR - 1) * p.gamma;
          double emin = fmin(e0, e1), emax = fmax(e0, e1);
          double lo = (PPAD - 1 - emax) / p.beta, hi = (PPAD + W - emin) / p.beta;
          if (lo > hi) { double t = lo; lo = hi; hi = t; }
          int jl = max((int)floor(lo), max(0, -p.bbase));
          int jh = min((int)ceil(hi), min(PACC - 1, J.nb - 1 - p.bbase));
          jlo[a] = jl;
          cnt[a] = max(0, jh - jl + 1);
        }
        pre[a + 1] = pre[a] + cnt[a];
      }
      const int total = pre[PA];
      for (int pidx = tid; pidx < total; pidx += PTHREADS) {
        int a = 0;
#pragma unroll
        for (int q = 1; q < PA; ++q) a += (pidx >= pre[q]) ? 1 : 0;
        int pa = 0, ja = 0;
#pragma unroll
        for (int q = 0; q < PA; ++q) if (q == a) { pa = pre[q]; ja = jlo[q]; }
        const int j = ja + (pidx - pa);
        const AngleParam& p = prm[a];
        const float xi = (float)(p.xi0 + j * p.beta + db * p.gamma);
        const float g = (float)p.gamma;
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int i = 0; i < PR; ++i) {
          float xx = i == 0 ? xi : fmaf((float)i, g, xi);
          float f = __builtin_amdgcn_fractf(xx);   // xx > 0: truncation is the floor
          int c0 = (int)xx;
          float v0 = band[i * PLS + c0];
          float v1 = band[i * PLS + c0 + 1];
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

  // partial sums of this region, pre-scaled by the path length per step
  float* part = J.partial + ((size_t)achunk * G + region) * (PA * PACC);
  for (int i = tid; i < PA * PACC; i += PTHREADS) {
    int a = i / PACC;
    part[i] = a < na ? acc[i] * prm[a].scale : 0.f;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (atomicAdd(&J.ticket[achunk], 1u) == (unsigned)(G - 1));
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  // last region of this angle chunk: add all regions' partials in order
  for (int i = tid; i < G * PA; i += PTHREADS) {
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
  const float* pbase = J.partial + (size_t)achunk * G * (PA * PACC);
  for (int idx = tid; idx < na * J.nb; idx += PTHREADS) {
    int a = idx / J.nb, b = idx - a * J.nb;
    float s = 0.f;
    for (int g = 0; g < G; ++g) {
      int j = b - fin_bbase[g * PA + a];
      if (j >= 0 && j < PACC) s += pbase[((size_t)g * PA + a) * PACC + j];
    }
    s *= J.scale;
    size_t o = (size_t)(a0 + a) * J.nb + b;
    J.out[o] = J.d ? s - J.d[o] : s;
  }
  if (tid == 0) J.ticket[achunk] = 0u;
}

template __global__ void k_project<Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project<Many<ProjJob>>(Many<ProjJob>);

}  // namespace tomo
