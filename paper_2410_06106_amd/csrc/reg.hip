// Regularization block of decentralized ADMM (the extra sub-problem that the
// paper's discussion proposes), for gfx950.  For every block (one per slice):
//   v = x - nu / rho_z,
//   z = prox_{theta R}(v),  theta = mu / rho_z,
//   t_z = z + nu / rho_z      (the block's target in the x-update),
// R Tikhonov (z = v / (1 + theta)) or isotropic total variation with forward
// differences that vanish across the last row / column, its prox by
// Chambolle's dual projection iterations
//   w = div p - v / theta,  p <- (p + tau grad w) / (1 + tau |grad w|),
//   z = v - theta div p.
// One thread per pixel; an iteration reads the field p of one slot and writes
// the other (neighbours read the old field), so a block alternates between the
// caller's field (slot 0) and a scratch one (slot 1); an odd iteration count
// starts from a copy in slot 1, so the last iteration always lands in slot 0.
// These kernels stream a few arrays per pixel and are bound by HBM.
#include "common.h"

namespace tomo {

namespace {

struct Field {
  const float* p1;
  const float* p2;
  int n;
  // (div p)(r, c) = p1(r, c) [r < n-1] - p1(r-1, c) [r > 0] + p2(r, c) [c < n-1] - p2(r, c-1) [c > 0]
  __device__ __forceinline__ float div(int r, int c) const {
    const size_t i = (size_t)r * n + c;
    float d = 0.f;
    if (r < n - 1) d += p1[i];
    if (r > 0) d -= p1[i - n];
    if (c < n - 1) d += p2[i];
    if (c > 0) d -= p2[i - 1];
    return d;
  }
};

__device__ __forceinline__ int slot_in(const RegJob& J, int t) { return (t + (J.iters & 1)) & 1; }

}  // namespace

// v, and for Tikhonov the whole z-update; for TV with an odd iteration count
// the copy of the field into slot 1
__global__ __launch_bounds__(256) void k_reg_init(Many<RegJob> src) {
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  const size_t cnt = (size_t)J.n * J.n;
  const size_t i = (size_t)lid * 256 + threadIdx.x;
  if (i >= cnt) return;
  const float nv = J.nu[i];
  const float v = J.x[i] - nv * J.irho_z;
  if (J.kind == REG_TIKHONOV) {
    const float z = v / (1.f + J.theta);
    J.z[i] = z;
    J.tz[i] = z + nv * J.irho_z;
    return;
  }
  J.tz[i] = v;
  if (J.iters & 1) {
    J.p[1][i] = J.p[0][i];
    J.p[1][cnt + i] = J.p[0][cnt + i];
  }
}

// Chambolle iteration t of every TV block that has more than t iterations
__global__ __launch_bounds__(256) void k_tv_iter(Many<RegJob> src, int t) {
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  if (J.kind != REG_TV || t >= J.iters) return;
  const int n = J.n;
  const size_t cnt = (size_t)n * n;
  const size_t i = (size_t)lid * 256 + threadIdx.x;
  if (i >= cnt) return;
  const int r = (int)(i / n), c = (int)(i - (size_t)r * n);
  const float* in = J.p[slot_in(J, t)];
  float* out = J.p[slot_in(J, t + 1)];
  const Field P{in, in + cnt, n};
  const float* v = J.tz;
  const float w = P.div(r, c) - v[i] / J.theta;
  float g1 = 0.f, g2 = 0.f;
  if (r < n - 1) g1 = (P.div(r + 1, c) - v[i + n] / J.theta) - w;
  if (c < n - 1) g2 = (P.div(r, c + 1) - v[i + 1] / J.theta) - w;
  const float den = 1.f + J.tau * sqrtf(g1 * g1 + g2 * g2);
  out[i] = (in[i] + J.tau * g1) / den;
  out[cnt + i] = (in[cnt + i] + J.tau * g2) / den;
}

// z = v - theta div p, t_z = z + nu / rho_z (TV blocks)
__global__ __launch_bounds__(256) void k_tv_final(Many<RegJob> src) {
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  if (J.kind != REG_TV) return;
  const int n = J.n;
  const size_t cnt = (size_t)n * n;
  const size_t i = (size_t)lid * 256 + threadIdx.x;
  if (i >= cnt) return;
  const int r = (int)(i / n), c = (int)(i - (size_t)r * n);
  const Field P{J.p[0], J.p[0] + cnt, n};
  const float z = J.tz[i] - J.theta * P.div(r, c);
  J.z[i] = z;
  J.tz[i] = z + J.nu[i] * J.irho_z;
}

}  // namespace tomo
