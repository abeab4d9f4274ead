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
// A workgroup owns an 8 x 56 tile.  A launch stages the tile's field and v
// with a halo of 4 pixels (a 16 x 64 region, one column per lane) in LDS and
// runs up to 4 iterations there (temporal blocking).  A launch reads the field of one slot and writes the other, since
// neighbouring tiles read the old field; a block alternates between the
// caller's field (slot 0) and a scratch one (slot 1), and an odd launch count
// starts from a copy in slot 1, so that the last launch lands in slot 0.  Per
// launch HBM moves the region's field and v (about 2.3 times the tile) in and
// the tile's field out, instead of 20 bytes per pixel for every iteration.
// The update divides by 1 + tau |grad w| with the hardware reciprocal and
// square root (each within about one unit in the last place).
#include "consensus.h"

namespace tomo {

namespace {

constexpr int TH = TV_TILE_H, TW = TV_TILE_W;    // tile; with its halo a 16 x 64 region
constexpr int TT = 256;

// field slot read by launch l of a block: the launches alternate slots and the
// last one writes slot 0 (an odd launch count starts from a copy in slot 1)
__device__ __forceinline__ int launches(const RegJob& J) { return (J.iters + TV_BLOCK - 1) / TV_BLOCK; }
__device__ __forceinline__ int slot_in(const RegJob& J, int l) { return (l + (launches(J) & 1)) & 1; }

struct Tile {
  int r0, c0;
};

__device__ __forceinline__ Tile tile_of(const RegJob& J, int lid) {
  const int tx = (J.n + TW - 1) / TW;
  const int ty = lid / tx;
  return Tile{ty * TH, (lid - ty * tx) * TW};
}

// (div p)(r, c) from the global field: p1(r, c) [r < n-1] - p1(r-1, c) [r > 0]
// + p2(r, c) [c < n-1] - p2(r, c-1) [c > 0]
__device__ __forceinline__ float div_global(const float* p1, const float* p2, int n, int r, int c) {
  const size_t i = (size_t)r * n + c;
  float d = 0.f;
  if (r < n - 1) d += p1[i];
  if (r > 0) d -= p1[i - n];
  if (c < n - 1) d += p2[i];
  if (c > 0) d -= p2[i - 1];
  return d;
}

}  // namespace

// v, and for Tikhonov the whole z-update; for TV with an odd iteration count
// the copy of the field into slot 1
__global__ __launch_bounds__(TT) void k_reg_init(Many<RegJob> src) {
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  const Tile T = tile_of(J, lid);
  const int n = J.n;
  const size_t cnt = (size_t)n * n;
  for (int k = threadIdx.x; k < TH * TW; k += TT) {
    const int r = T.r0 + k / TW, c = T.c0 + k % TW;
    if (r >= n || c >= n) continue;
    const size_t i = (size_t)r * n + c;
    const float nv = J.nu[i];
    const float v = J.x[i] - nv * J.irho_z;
    if (J.kind == REG_TIKHONOV) {
      const float z = v / (1.f + J.theta);
      J.z[i] = z;
      J.tz[i] = z + nv * J.irho_z;
      continue;
    }
    J.tz[i] = v;
    if (launches(J) & 1) {
      J.p[1][i] = J.p[0][i];
      J.p[1][cnt + i] = J.p[0][cnt + i];
    }
  }
}

// Chambolle iterations [t0, t0 + k) of every TV block that has more than t0
// iterations, k = min(TV_BLOCK, remaining): the tile and a halo of TV_BLOCK
// pixels are staged in LDS and iterated there.  Each iteration is exact on the
// region shrunk by one pixel per side (a value depends on its neighbours at
// distance one), so after k <= TV_BLOCK iterations the tile is exact; in-image
// values never depend on values outside the image (the zero-flux conditions),
// so the halo is simply cut at the image border.
__global__ __launch_bounds__(TT) void k_tv_iter(Many<RegJob> src, int t0) {
  constexpr int H = TV_BLOCK, RH = TH + 2 * H, RW = TW + 2 * H, RN = RH * RW;
  constexpr int RPT = RN / TT;                     // region rows per thread
  static_assert(RW == 64 && RN % TT == 0, "a thread owns one region column");
  __shared__ float s1[RN], s2[RN], sv[RN], sw[RN];
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  if (J.kind != REG_TV || t0 >= J.iters) return;
  const int kk = min(H, J.iters - t0);
  const Tile T = tile_of(J, lid);
  const int n = J.n, R0 = T.r0 - H, C0 = T.c0 - H;
  const size_t cnt = (size_t)n * n;
  const int launch = t0 / H;
  // slot pointers by select, not by a runtime index into J.p (which would put
  // the job in scratch memory)
  const bool s_in = slot_in(J, launch) != 0;
  const float* p1 = s_in ? J.p[1] : J.p[0];
  float* o1 = s_in ? J.p[0] : J.p[1];
  const float ith = 1.f / J.theta, tau = J.tau;
  // thread: region column cl, rows rb, rb + TT/64, ...
  const int cl = threadIdx.x & 63, rb = threadIdx.x >> 6, c = C0 + cl;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int rl = rb + j * (TT / 64), r = R0 + rl, k = rl * RW + cl;
    const bool in = r >= 0 && r < n && c >= 0 && c < n;
    const size_t i = in ? (size_t)r * n + c : 0;
    s1[k] = in ? p1[i] : 0.f;
    s2[k] = in ? p1[cnt + i] : 0.f;
    sv[k] = in ? J.tz[i] * ith : 0.f;          // v / theta
  }
  __syncthreads();
  for (int it = 0; it < kk; ++it) {
    // w = div p - v / theta (neighbours outside the region read as zero: only the
    // stale ring is affected)
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int rl = rb + j * (TT / 64), r = R0 + rl, k = rl * RW + cl;
      float d = 0.f;
      if (r < n - 1) d += s1[k];
      if (r > 0 && rl > 0) d -= s1[k - RW];
      if (c < n - 1) d += s2[k];
      if (c > 0 && cl > 0) d -= s2[k - 1];
      sw[k] = d - sv[k];
    }
    __syncthreads();
    // p <- (p + tau grad w) / (1 + tau |grad w|), in place (a value reads only itself and w)
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int rl = rb + j * (TT / 64), r = R0 + rl, k = rl * RW + cl;
      const float w = sw[k];
      const float g1 = (r < n - 1 && rl < RH - 1) ? sw[k + RW] - w : 0.f;
      const float g2 = (c < n - 1 && cl < RW - 1) ? sw[k + 1] - w : 0.f;
      const float inv = __builtin_amdgcn_rcpf(fmaf(tau, __builtin_amdgcn_sqrtf(g1 * g1 + g2 * g2), 1.f));
      s1[k] = (s1[k] + tau * g1) * inv;
      s2[k] = (s2[k] + tau * g2) * inv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int rl = rb + j * (TT / 64), r = R0 + rl;
    if (rl < H || rl >= H + TH || cl < H || cl >= H + TW || r >= n || c >= n) continue;
    const size_t i = (size_t)r * n + c;
    o1[i] = s1[rl * RW + cl];
    o1[cnt + i] = s2[rl * RW + cl];
  }
}

// z = v - theta div p, t_z = z + nu / rho_z (TV blocks)
__global__ __launch_bounds__(TT) void k_tv_final(Many<RegJob> src) {
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  if (J.kind != REG_TV) return;
  const Tile T = tile_of(J, lid);
  const int n = J.n;
  const size_t cnt = (size_t)n * n;
  const float* p1 = J.p[0];
  for (int k = threadIdx.x; k < TH * TW; k += TT) {
    const int r = T.r0 + k / TW, c = T.c0 + k % TW;
    if (r >= n || c >= n) continue;
    const size_t i = (size_t)r * n + c;
    const float z = J.tz[i] - J.theta * div_global(p1, p1 + cnt, n, r, c);
    J.z[i] = z;
    J.tz[i] = z + J.nu[i] * J.irho_z;
  }
}

}  // namespace tomo
