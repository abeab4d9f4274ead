// Forward projector d = P u (Eq. 2-4) for gfx950, region-resident form:
// Joseph ray-driven interpolation with one image region held in LDS for all
// angles of a node.
//
// A workgroup owns one 128 x 128 region of one node's image and every angle of
// that node.  It stages the region in LDS once per angle class (rows for
// row-driven angles, columns transposed for column-driven ones), then its
// waves take work items -- one angle and 64 consecutive rays -- from a shared
// counter until none are left: no barrier separates the items.  A lane walks
// its ray through the region line by line in unrolled bands of 32 lines,
// skipping bands that none of the item's rays meets; positions outside the
// region are clamped onto the two zero samples on either side of the line, so
// every read stays in the region's LDS lines.  Each item writes the partial ray sums of its 64 rays for this
// region; a second launch adds the regions' partials in region order, so the
// result does not depend on which wave ran which item (bit-reproducible).
#include "common.h"

namespace tomo {

namespace {

struct QAngle {
  double xi0;     // interpolation coordinate of ray 0 at driving line 0 (LDS units)
  double beta;    // d(xi)/d(ray)
  double gamma;   // d(xi)/d(line)
  double rlo0;    // first candidate ray of a band starting at line 0 (affine in the band start)
  double rhi0;    // last candidate ray of such a band
  double rsl;     // slope of both with the band start
  float scale;    // path length per step: 1/|cos| or 1/|sin|
  float g32;      // gamma rounded to float32
  int jlo, jhi;   // rays of this region that land on detector bins (inclusive)
};

__device__ __forceinline__ void region_geom(const ProjJob& J, int region, int& gr0, int& gc0, int& gh, int& gw) {
  const int rr = region / J.n_rc, rc = region - rr * J.n_rc;
  gr0 = rr * J.reg_h;
  gc0 = rc * J.reg_w;
  gh = min(J.reg_h, J.n - gr0);
  gw = min(J.reg_w, J.n - gc0);
}

// Detector bins the region's pixels can touch for angle (cs, sn): floor of
// the smallest and largest bin coordinate over the region corners; a pixel
// touches floor(s) and floor(s) + 1.
__device__ __forceinline__ void region_bins(double cs, double sn, double h, double hb, int gr0, int gc0, int gh,
                                            int gw, int& bbase, int& nray) {
  const double s00 = (gc0 - h) * cs + (gr0 - h) * sn + hb;
  const double dc = (gw - 1) * cs, dr = (gh - 1) * sn;
  bbase = (int)floor(s00 + fmin(0.0, dc) + fmin(0.0, dr));
  const int btop = (int)floor(s00 + fmax(0.0, dc) + fmax(0.0, dr)) + 1;
  nray = btop - bbase + 1;
}

__device__ __forceinline__ bool row_driven(double cs, double sn) { return fabs(cs) >= fabs(sn); }

}  // namespace

template <class Src>
__global__ __launch_bounds__(QTHREADS) void k_project_res(Src src) {
  __shared__ __align__(16) float reg[QR * QLS];
  __shared__ QAngle prm[QAG];
  __shared__ int cstart[QAG + 1];
  __shared__ int next_item;

  int lid;
  const ProjJob J = src.get(blockIdx.x, lid);
  const int G = J.n_rr * J.n_rc;
  const int region = lid;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  constexpr int NW = QTHREADS / 64;
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);
  int gr0, gc0, gh, gw;
  region_geom(J, region, gr0, gc0, gh, gw);

  for (int cls = 0; cls < 2; ++cls) {
    int any = 0;
    for (int a = tid; a < J.n_ang; a += QTHREADS) {
      const double th = J.ang[a];
      any |= (row_driven(cos(th), sin(th)) ? 0 : 1) == cls;
    }
    if (!__syncthreads_or(any)) continue;
    const int D = cls == 0 ? gh : gw;   // driving lines
    const int W = cls == 0 ? gw : gh;   // samples per line

    // stage the region: line i, sample k at reg[i * QLS + QOFF + k]; the two
    // samples on each side of a line and unused lines stay zero
    for (int i = tid; i < QR * 4; i += QTHREADS) {   // the two samples on each side of every line
      const int line = i >> 2, q = i & 3;
      reg[line * QLS + (q < 2 ? q : W + QOFF + q - 2)] = 0.f;
    }
    for (int i = D * QLS + tid; i < QR * QLS; i += QTHREADS) reg[i] = 0.f;   // unused lines
    if (cls == 0) {
      for (int idx = tid; idx < gh * gw; idx += QTHREADS) {
        const int i = idx / gw, k = idx - i * gw;
        reg[i * QLS + QOFF + k] = J.img[(size_t)(gr0 + i) * J.n + gc0 + k];
      }
    } else {
      // lane -> image row k (consecutive LDS addresses), waves over columns
      for (int k0 = 0; k0 < gh; k0 += 64) {
        const int k = k0 + lane;
        if (k < gh)
          for (int i = wave; i < gw; i += NW) reg[i * QLS + QOFF + k] = J.img[(size_t)(gr0 + k) * J.n + gc0 + i];
      }
    }

    for (int a0 = 0; a0 < J.n_ang; a0 += QAG) {
      const int na = min(QAG, J.n_ang - a0);
      __syncthreads();       // staging done / previous group's items finished
      if (tid < QAG) {
        QAngle p{};
        p.jlo = 0;
        p.jhi = -1;
        if (tid < na) {
          const double th = J.ang[a0 + tid];
          const double cs = cos(th), sn = sin(th);
          if ((row_driven(cs, sn) ? 0 : 1) == cls) {
            int bbase, nray;
            region_bins(cs, sn, h, hb, gr0, gc0, gh, gw, bbase, nray);
            double ib;
            if (cls == 0) {
              p.beta = 1.0 / cs;
              ib = cs;
              p.gamma = -sn / cs;
              p.xi0 = (bbase - hb - (gr0 - h) * sn) / cs + h - gc0 + QOFF;
              p.scale = (float)(1.0 / fabs(cs));
            } else {
              p.beta = 1.0 / sn;
              ib = sn;
              p.gamma = -cs / sn;
              p.xi0 = (bbase - hb - (gc0 - h) * cs) / sn + h - gr0 + QOFF;
              p.scale = (float)(1.0 / fabs(sn));
            }
            // rays j with QOFF-1 < xi(j, line) < QOFF+W for some line of a
            // 32-line band starting at line db: affine bounds in db
            const double span = (QBAND - 1) * p.gamma;
            const double t1 = (QOFF - 1 - p.xi0 - fmax(0.0, span)) * ib;
            const double t2 = (QOFF + W - p.xi0 - fmin(0.0, span)) * ib;
            p.rlo0 = fmin(t1, t2);
            p.rhi0 = fmax(t1, t2);
            p.rsl = -p.gamma * ib;
            p.g32 = (float)p.gamma;
            p.jlo = max(0, -bbase);
            p.jhi = min(min(nray, QACC) - 1, J.nb - 1 - bbase);
          }
        }
        prm[tid] = p;
      }
      __syncthreads();
      if (tid == 0) {
        int c = 0;
        for (int a = 0; a < QAG; ++a) {
          cstart[a] = c;
          const int nr = prm[a].jhi - prm[a].jlo + 1;
          c += nr > 0 ? (nr + 63) >> 6 : 0;
        }
        cstart[QAG] = c;
        next_item = 0;
      }
      __syncthreads();
      const int total = cstart[QAG];

      // items: one angle and 64 consecutive rays, taken by waves as they free up
      for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(&next_item, 1);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0, 64));
        if (it >= total) break;
        int a = 0;
        for (int step = QAG / 2; step > 0; step >>= 1)   // largest a with cstart[a] <= it
          if (cstart[a + step] <= it) a += step;
        const QAngle& p = prm[a];
        const int j0 = p.jlo + ((it - cstart[a]) << 6);
        const int j = j0 + lane;
        const float g = p.g32;
        float s0 = 0.f, s1 = 0.f;
        for (int db = 0; db < D; db += QBAND) {
          const int jl = (int)floor(p.rlo0 + db * p.rsl);
          const int jh = (int)ceil(p.rhi0 + db * p.rsl);
          if (jh < j0 || jl > j0 + 63) continue;           // no ray of the item meets this band
          const float xi = (float)(p.xi0 + db * p.gamma + (double)j * p.beta);
          const float* base = reg + db * QLS;
#pragma unroll
          for (int i = 0; i < QBAND; ++i) {
            const float xx = i == 0 ? xi : fmaf((float)i, g, xi);
            const float f = __builtin_amdgcn_fractf(xx);
            const int c0 = min(max((int)xx, 0), W + QOFF);     // off the region: two zero samples
            const float v0 = base[i * QLS + c0];
            const float v1 = base[i * QLS + c0 + 1];
            s0 += v0;
            s1 = fmaf(f, v1 - v0, s1);
          }
        }
        if (j <= p.jhi) J.partial[((size_t)(a0 + a) * G + region) * QACC + j] = (s0 + s1) * p.scale;
      }
    }
    __syncthreads();         // every item done before the region is restaged
  }
}

// out = scale * sum over regions of the partial ray sums - d, regions added
// in region order; one thread per (angle, bin), a workgroup per angle and
// block of QTHREADS bins.
template <class Src>
__global__ __launch_bounds__(QTHREADS) void k_project_res_reduce(Src src) {
  __shared__ int rb[PMAXREG], rn[PMAXREG];
  int lid;
  const ProjJob J = src.get(blockIdx.x, lid);
  const int G = J.n_rr * J.n_rc;
  const int nbb = (J.nb + QTHREADS - 1) / QTHREADS;
  const int a = lid / nbb;
  const int b = (lid - a * nbb) * QTHREADS + threadIdx.x;
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);
  const double th = J.ang[a];
  const double cs = cos(th), sn = sin(th);
  for (int g = threadIdx.x; g < G; g += QTHREADS) {
    int gr0, gc0, gh, gw, bbase, nray;
    region_geom(J, g, gr0, gc0, gh, gw);
    region_bins(cs, sn, h, hb, gr0, gc0, gh, gw, bbase, nray);
    rb[g] = bbase;
    rn[g] = min(nray, QACC);
  }
  __syncthreads();
  if (b >= J.nb) return;
  const float* pa = J.partial + (size_t)a * G * QACC;
  float s = 0.f;
  for (int g = 0; g < G; ++g) {
    const int j = b - rb[g];
    if (j >= 0 && j < rn[g]) s += pa[(size_t)g * QACC + j];
  }
  const size_t o = (size_t)a * J.nb + b;
  const float v = s * J.scale;
  J.out[o] = J.d ? v - J.d[o] : v;
}

template __global__ void k_project_res<Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project_res<Many<ProjJob>>(Many<ProjJob>);
template __global__ void k_project_res_reduce<Single<ProjJob>>(Single<ProjJob>);
template __global__ void k_project_res_reduce<Many<ProjJob>>(Many<ProjJob>);

}  // namespace tomo
