// Matched backprojector P^T (the exact transpose of the Joseph projector) for
// gfx950, voxel-driven: every thread gathers for 4 adjacent pixels of a 32x32
// tile.  For each angle the two detector bins a pixel touches (Eq. 2-4 closed
// form: weight max(0, 1 - |t_b - t_rc| / c) / c on bins floor(s), floor(s)+1)
// are read from a 48-bin window of the sinogram row staged in LDS and pre-scaled
// by 1/c, so a pixel-angle update costs two clamped weights and two FMAs.
// Gather only: no atomics, bit-reproducible.  The chord-length model (CHORD)
// uses the same two bins with the trapezoid weight of the pixel's chord
// instead of the triangle, positions in float64.  Epilogues: plain
// (image = alpha P^T s + beta image) or the u-step of Alg. 2
// (u -= eta1 (P^T r + rho (u - x) + lambda)).
#include "common.h"

namespace tomo {

template <class Src, bool CHORD>
__global__ __launch_bounds__(BTHREADS) void k_backproject(Src src) {
  __shared__ float sw[BAC * BW];
  __shared__ float4 aprm[BAC];
  __shared__ int wbase[BAC];
  // chord lengths only: cos, sin, the tile origin's window coordinate and the
  // trapezoid's outer half-width w2 in float64 (the ramp can be far narrower
  // than a float32 rounding of w2), 1 / (w2 - w1), and for an axis-aligned
  // angle the orientation of the half-open pixel convention
  __shared__ double4 cprm[CHORD ? BAC : 1];
  __shared__ float tprm[CHORD ? BAC : 1];
  __shared__ int axis[CHORD ? BAC : 1];

  int lid;
  const BPJob J = src.get(blockIdx.x, lid);
  const int ty = lid / J.tiles_x, tx = lid - ty * J.tiles_x;
  const int r0 = ty * BT, c0 = tx * BT;
  const int tid = threadIdx.x;
  const int dy = tid >> 3, dx0 = (tid & 7) * 4;
  const double h = 0.5 * (J.n - 1), hb = 0.5 * (J.nb - 1);

  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;

  for (int ac = 0; ac < J.n_ang; ac += BAC) {
    const int nac = min(BAC, J.n_ang - ac);
    __syncthreads();
    if (tid < nac) {
      double cs, sn;
      angle_trig(J.ang[ac + tid], CHORD, cs, sn);
      double s00 = (c0 - h) * cs + (r0 - h) * sn + hb;     // bin coordinate of the tile origin
      double dc = (BT - 1) * cs, dr = (BT - 1) * sn;
      int wb = (int)floor(s00 + fmin(0.0, dc) + fmin(0.0, dr)) - 1;
      double c = fmax(fabs(cs), fabs(sn));
      aprm[tid] = make_float4((float)cs, (float)sn, (float)(s00 - wb), (float)(1.0 / c));
      wbase[tid] = wb;
      if (CHORD) {
        const double w1 = 0.5 * fabs(fabs(cs) - fabs(sn)), w2 = 0.5 * (fabs(cs) + fabs(sn));
        cprm[tid] = make_double4(cs, sn, s00 - wb, w2);
        tprm[tid] = w2 > w1 ? (float)(1.0 / (w2 - w1)) : 0.f;
        // axis-aligned: +1 when the line's coordinate grows with t, else -1
        axis[tid] = sn == 0.0 ? (cs > 0.0 ? 1 : -1) : (cs == 0.0 ? (sn > 0.0 ? 1 : -1) : 0);
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nac * BW; idx += BTHREADS) {
      int a = idx / BW, k = idx - a * BW;
      int b = wbase[a] + k;
      float v = (b >= 0 && b < J.nb) ? J.sino[(size_t)(ac + a) * J.nb + b] : 0.f;
      sw[idx] = v * aprm[a].w;
    }
    __syncthreads();
    if (CHORD) {
      for (int a = 0; a < nac; ++a) {
        const double4 p = cprm[a];
        const float invr = tprm[a];
        const int ax = axis[a];
        const float* row = sw + a * BW;
        const double sb = fma((double)dy, p.y, fma((double)dx0, p.x, p.z));
        float* accs[4] = {&acc0, &acc1, &acc2, &acc3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double sd = q == 0 ? sb : fma((double)q, p.x, sb);
          const int b0 = (int)sd;                        // window coordinates are >= 0
          const double f = sd - (double)b0;              // |D| to bin b0; 1 - f to bin b0 + 1
          float w0, w1;
          if (ax != 0) {                                 // half-open pixels
            w0 = (ax > 0 ? f <= 0.5 : f < 0.5) ? 1.f : 0.f;
            w1 = 1.f - w0;
          } else {
            w0 = __builtin_amdgcn_fmed3f((float)(p.w - f) * invr, 0.f, 1.f);
            w1 = __builtin_amdgcn_fmed3f((float)(p.w - 1.0 + f) * invr, 0.f, 1.f);
          }
          *accs[q] = fmaf(w0, row[b0], *accs[q]);
          *accs[q] = fmaf(w1, row[b0 + 1], *accs[q]);
        }
      }
      continue;
    }
    for (int a = 0; a < nac; ++a) {
      const float4 p = aprm[a];
      const float gam = p.w, omg = 1.f - p.w;
      const float* row = sw + a * BW;
      const float sb = fmaf((float)dy, p.y, fmaf((float)dx0, p.x, p.z));
      // window coordinates are >= 0, so truncation is the floor
#define TOMO_BP_STEP(Q, ACC)                                           \
      {                                                                \
        float s = (Q) == 0 ? sb : fmaf((float)(Q), p.x, sb);           \
        float f = __builtin_amdgcn_fractf(s);                          \
        int b0 = (int)s;                                               \
        float v0 = row[b0], v1 = row[b0 + 1];                          \
        float w0 = __builtin_amdgcn_fmed3f(fmaf(-f, gam, 1.f), 0.f, 1.f); \
        float w1 = __builtin_amdgcn_fmed3f(fmaf(f, gam, omg), 0.f, 1.f);  \
        ACC = fmaf(w0, v0, ACC);                                       \
        ACC = fmaf(w1, v1, ACC);                                       \
      }
      TOMO_BP_STEP(0, acc0)
      TOMO_BP_STEP(1, acc1)
      TOMO_BP_STEP(2, acc2)
      TOMO_BP_STEP(3, acc3)
#undef TOMO_BP_STEP
    }
  }

  const int r = r0 + dy;
  if (r >= J.n) return;
  const int cb = c0 + dx0;
  float accv[4] = {acc0, acc1, acc2, acc3};
  float* out = J.img + (size_t)r * J.n;
  if (J.mode == BP_PLAIN) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int c = cb + q;
      if (c < J.n) out[c] = J.beta != 0.f ? fmaf(J.alpha, accv[q], J.beta * out[c]) : J.alpha * accv[q];
    }
  } else {
    // ADMM u-step, in place (BP_ADMM) or from u_in with (rho, eta1) read
    // from device memory (BP_UNROLL)
    const float* xr = J.x + (size_t)r * J.n;
    const float* lr = J.lam + (size_t)r * J.n;
    const float* ur = J.u_in ? J.u_in + (size_t)r * J.n : out;
    const float rho = J.scal ? J.scal[0] : J.rho, eta = J.scal ? J.scal[1] : J.eta1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int c = cb + q;
      if (c < J.n) {
        float u = ur[c];
        float g = accv[q] + fmaf(rho, u - xr[c], lr[c]);
        out[c] = fmaf(-eta, g, u);
      }
    }
  }
}

template __global__ void k_backproject<Single<BPJob>, false>(Single<BPJob>);
template __global__ void k_backproject<Many<BPJob>, false>(Many<BPJob>);
template __global__ void k_backproject<Single<BPJob>, true>(Single<BPJob>);
template __global__ void k_backproject<Many<BPJob>, true>(Many<BPJob>);

}  // namespace tomo
