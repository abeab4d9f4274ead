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
// A workgroup of 1024 threads owns a 20 x 52 tile.  One z-update of a TV block
// is an even number of launches of k_reg_step; each stages the tile's field
// with a halo of 6 pixels (a 32 x 64 region, one column per lane, two rows per
// thread) in LDS, forms v there from x and nu, and runs up to 6 iterations on
// it (temporal blocking).  A
// launch reads the field of one slot and writes the other, since neighbouring
// tiles read the old field; the launches alternate between the caller's field
// (slot 0) and a scratch one (slot 1), starting from slot 0 and, their count
// being even, ending in it.  The last launch runs at most 5 iterations, so that
// the field one pixel above and left of its tile is exact as well, and forms z
// and t_z from the divergence in LDS.  Nothing but z and t_z is written outside
// the field, so the launches need no other pass over the image.  The update
// divides by 1 + tau |grad w| with the hardware reciprocal and square root
// (each within about one unit in the last place).
#include "consensus.h"

namespace tomo {

namespace {

constexpr int TH = TV_TILE_H, TW = TV_TILE_W;    // tile; with its halo a 32 x 64 region
constexpr int TT = TV_THREADS;

struct Tile {
  int r0, c0;
};

__device__ __forceinline__ Tile tile_of(const RegJob& J, int lid) {
  const int tx = (J.n + TW - 1) / TW;
  const int ty = lid / tx;
  return Tile{ty * TH, (lid - ty * tx) * TW};
}

__device__ __forceinline__ float v_of(const RegJob& J, size_t i) { return J.x[i] - J.nu[i] * J.irho_z; }

}  // namespace

// Launch l of the z-update of every block.  Tikhonov blocks finish in launch 0.
// A TV block with T iterations takes L = tv_launches(T) launches; launch l runs
// tv_launch_iters(T, L, l) of them from the field in slot (L - l) & 1 (slot 0
// when T = 0) into the other slot.  Each iteration is exact on the region
// shrunk by one pixel per side (a value depends on its neighbours at distance
// one), so after k <= 6 iterations the tile is exact, and after k <= 5 so is
// the ring around it; in-image values never depend on values outside the image
// (the zero-flux conditions), so the halo is simply cut at the image border.
__global__ __launch_bounds__(TT) void k_reg_step(Many<RegJob> src, int l) {
  constexpr int H = TV_BLOCK, RH = TH + 2 * H, RW = TW + 2 * H, RN = RH * RW;
  constexpr int RPT = RN / TT;                     // region rows per thread
  static_assert(RW == 64 && RN % TT == 0, "a thread owns one region column");
  __shared__ float s1[RN], s2[RN], sv[RN], sw[RN];
  int lid;
  const RegJob J = src.get(blockIdx.x, lid);
  const Tile T = tile_of(J, lid);
  const int n = J.n;
  if (J.kind == REG_TIKHONOV) {
    if (l != 0) return;
    for (int k = threadIdx.x; k < TH * TW; k += TT) {
      const int r = T.r0 + k / TW, c = T.c0 + k % TW;
      if (r >= n || c >= n) continue;
      const size_t i = (size_t)r * n + c;
      const float z = v_of(J, i) / (1.f + J.theta);
      J.z[i] = z;
      J.tz[i] = z + J.nu[i] * J.irho_z;
    }
    return;
  }
  const int L = tv_launches(J.iters);
  if (l >= L) return;
  const int kk = tv_launch_iters(J.iters, L, l);
  const int R0 = T.r0 - H, C0 = T.c0 - H;
  const size_t cnt = (size_t)n * n;
  // slot pointers by select, not by a runtime index into J.p (which would put
  // the job in scratch memory)
  const bool s_in = J.iters > 0 && ((L - l) & 1) != 0;
  const float* p1 = s_in ? J.p[1] : J.p[0];
  float* o1 = s_in ? J.p[0] : J.p[1];
  const float ith = J.iters > 0 ? 1.f / J.theta : 0.f, tau = J.tau;
  // thread: region column cl, rows rb, rb + TT/64, ...
  const int cl = threadIdx.x & 63, rb = threadIdx.x >> 6, c = C0 + cl;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int rl = rb + j * (TT / 64), r = R0 + rl, k = rl * RW + cl;
    const bool in = r >= 0 && r < n && c >= 0 && c < n;
    const size_t i = in ? (size_t)r * n + c : 0;
    s1[k] = in ? p1[i] : 0.f;
    s2[k] = in ? p1[cnt + i] : 0.f;
    sv[k] = in ? v_of(J, i) * ith : 0.f;      // v / theta
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
  const bool last = l == L - 1;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int rl = rb + j * (TT / 64), r = R0 + rl, k = rl * RW + cl;
    if (rl < H || rl >= H + TH || cl < H || cl >= H + TW || r >= n || c >= n) continue;
    const size_t i = (size_t)r * n + c;
    if (J.iters > 0) {
      o1[i] = s1[k];
      o1[cnt + i] = s2[k];
    }
    if (last) {
      // z = v - theta div p; the neighbours above and to the left are exact (kk < TV_BLOCK)
      float d = 0.f;
      if (r < n - 1) d += s1[k];
      if (r > 0) d -= s1[k - RW];
      if (c < n - 1) d += s2[k];
      if (c > 0) d -= s2[k - 1];
      const float nv = J.nu[i];
      const float z = (J.x[i] - nv * J.irho_z) - J.theta * d;
      J.z[i] = z;
      J.tz[i] = z + nv * J.irho_z;
    }
  }
}

}  // namespace tomo
