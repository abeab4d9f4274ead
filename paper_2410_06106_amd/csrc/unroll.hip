// Elementwise steps of the unrolled (differentiable) decentralized ADMM and
// their exact backward passes, for gfx950.  With the nodes' images stacked as
// [M][npix] (npix = n * n) and the penalty and step of an iteration held in
// device memory (so that learned values never reach the host):
//
//   u-step (Alg. 2)     U' = U - eta (B + rho (U - x) + L),  B = P^T (P U - D)
//   x-update SEG (Alg. 3, E2 steps from x on the segment each node owns)
//                       x' = t + a^E2 (x - t),  t = U_o + L_o / rho,  a = 1 - eta2 rho
//                       (o = the owner of the pixel's row; E2 steps of a linear recurrence,
//                       evaluated in this closed form as x + (1 - a^E2)(t - x))
//   x-update AVG (Eq. 9) x' = (1/M) sum_m (U_m + L_m / rho)
//   dual (Eq. 24)       L' = L + rho (U - x')
//
// Backward passes take the gradient G of a step's output and return the
// gradients of its tensor inputs and of (rho, eta).  The scalar gradients are
// sums over every pixel of every node: each workgroup reduces its share in
// float64 into a partial, and a one-workgroup finish kernel adds the partials in
// a fixed order (results do not depend on scheduling) and forms the scalars.
#include "common.h"

namespace tomo {

namespace {

constexpr int UT = 256;          // threads per workgroup

// float64 workgroup sum of up to three values into part[blockIdx.x * 3 + i]
__device__ __forceinline__ void wg_sum3(double a, double b, double c, double* part) {
  __shared__ double red[3][UT / 64];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int i = 0; i < UT / 64; ++i) s += red[threadIdx.x][i];
    part[(size_t)blockIdx.x * 3 + threadIdx.x] = s;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// u-step
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(UT) void k_unroll_ustep(int m, long long npix, const float* U, const float* B,
                                                     const float* x, const float* L, const float* scal, float* Uo) {
  const float rho = scal[0], eta = scal[1];
  const long long total = (long long)m * npix;
  for (long long i = ((long long)blockIdx.x * UT + threadIdx.x); i < total; i += (long long)gridDim.x * UT) {
    const long long p = i % npix;
    Uo[i] = U[i] - eta * (B[i] + rho * (U[i] - x[p]) + L[i]);
  }
}

// Gradients of U' = U - eta (B + rho (U - x) + L) with B = P^T (P U - D):
//   dU = G - eta (P^T P G + rho G),  dL = -eta G,  dx = eta rho sum_m G_m,
//   d eta = -(<P G, R> + rho <G, U - x> + <G, L>),  d rho = -eta <G, U - x>,
// R = P U - D the forward residual.  One thread per pixel handles it for all
// nodes (so dx needs no atomics); part[wg] = (<G, U - x>, <G, L>, 0).  With
// acc, dL and dx are added to instead of written.
__global__ __launch_bounds__(UT) void k_unroll_ustep_grad(int m, long long npix, const float* G, const float* PtPG,
                                                          const float* U, const float* x, const float* L,
                                                          const float* scal, float* dU, float* dL, float* dx,
                                                          int acc, double* part) {
  const float rho = scal[0], eta = scal[1];
  double sux = 0.0, sl = 0.0;
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    const float xp = x[p];
    float gs = 0.f;
    for (int k = 0; k < m; ++k) {
      const long long i = (long long)k * npix + p;
      const float g = G[i];
      dU[i] = g - eta * (PtPG[i] + rho * g);
      dL[i] = acc ? fmaf(-eta, g, dL[i]) : -eta * g;
      gs += g;
      sux += (double)g * ((double)U[i] - (double)xp);
      sl += (double)g * (double)L[i];
    }
    dx[p] = acc ? fmaf(eta * rho, gs, dx[p]) : eta * rho * gs;
  }
  wg_sum3(sux, sl, 0.0, part);
}

// <a, b> over n values: part[wg] = (sum, 0, 0)
__global__ __launch_bounds__(UT) void k_unroll_dot(long long n, const float* a, const float* b, double* part) {
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * UT + threadIdx.x; i < n; i += (long long)gridDim.x * UT)
    s += (double)a[i] * (double)b[i];
  wg_sum3(s, 0.0, 0.0, part);
}

// ---------------------------------------------------------------------------
// x-update, SEG: owner[r] = node owning image row r
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(UT) void k_unroll_xseg(int n, const int* owner, const float* U, const float* L,
                                                    const float* x, const float* scal, float eta2, int e2,
                                                    float* xo) {
  const float rho = scal[0];
  const long long npix = (long long)n * n;
  double aE = 1.0;
  for (int e = 0; e < e2; ++e) aE *= 1.0 - (double)eta2 * rho;
  const float q = (float)(1.0 - aE);
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    const long long i = (long long)owner[p / n] * npix + p;
    const float t = U[i] + L[i] / rho;
    const float xs = x[p];
    xo[p] = e2 > 0 ? fmaf(q, t - xs, xs) : xs;
  }
}

// Gradients of x' = t + a^E2 (x - t), t = U_o + L_o / rho, a = 1 - eta2 rho:
//   dx = a^E2 G;  dU_o = (1 - a^E2) G;  dL_o = (1 - a^E2) G / rho (zero on the
//   rows a node does not own);  d rho = sum G ((1 - a^E2)(-L_o / rho^2)
//   - E2 eta2 a^(E2-1) (x - t)).  part[wg] = (d rho share, 0, 0).
__global__ __launch_bounds__(UT) void k_unroll_xseg_grad(int m, int n, const int* owner, const float* G,
                                                         const float* U, const float* L, const float* x,
                                                         const float* scal, float eta2, int e2, float* dU,
                                                         float* dL, float* dx, double* part) {
  const double rho = scal[0];
  const double a = 1.0 - (double)eta2 * rho;
  double aE = 1.0, aE1 = 1.0;                      // a^E2, a^(E2-1)
  for (int e = 0; e < e2; ++e) { aE1 = aE; aE *= a; }
  const long long npix = (long long)n * n;
  double sr = 0.0;
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    const int o = owner[p / n];
    const double g = G[p];
    const long long io = (long long)o * npix + p;
    const double lo = L[io], t = (double)U[io] + lo / rho;
    dx[p] = (float)(aE * g);
    for (int k = 0; k < m; ++k) {
      const long long i = (long long)k * npix + p;
      dU[i] = k == o ? (float)((1.0 - aE) * g) : 0.f;
      dL[i] = k == o ? (float)((1.0 - aE) * g / rho) : 0.f;
    }
    sr += g * ((1.0 - aE) * (-lo / (rho * rho)) - (double)e2 * eta2 * aE1 * ((double)x[p] - t));
  }
  wg_sum3(sr, 0.0, 0.0, part);
}

// Gradients of the SEG x-update followed by the dual update, (xs, Lo) with
// xs = t + a^E2 (x - t) and Lo = L + rho (U - xs), given Gx = dLoss/dxs (from
// later uses of xs) and GL = dLoss/dLo, in one pass: gx = Gx - rho sum_m GL_m
// is the total gradient of xs; dL = GL (+ (1 - a^E2) gx / rho on the owner's
// rows), dU = rho GL (+ (1 - a^E2) gx on the owner's rows), dx = a^E2 gx,
// d rho = sum_m <GL_m, U_m - xs> + the Alg. 3 term of gx.  part[wg] = (d rho share, 0, 0).
__global__ __launch_bounds__(UT) void k_unroll_segdual_grad(int m, int n, const int* owner, const float* Gx,
                                                            const float* GL, const float* U, const float* L,
                                                            const float* x, const float* xs, const float* scal,
                                                            float eta2, int e2, float* dU, float* dL, float* dx,
                                                            double* part) {
  const float rho_f = scal[0];
  const double rho = rho_f;
  const double a = 1.0 - (double)eta2 * rho;
  double aE = 1.0, aE1 = 1.0;                      // a^E2, a^(E2-1)
  for (int e = 0; e < e2; ++e) { aE1 = aE; aE *= a; }
  const long long npix = (long long)n * n;
  double sr = 0.0;
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    const int o = owner[p / n];
    float gs = 0.f;
    for (int k = 0; k < m; ++k) gs += GL[(long long)k * npix + p];
    const float gxf = Gx[p] + -rho_f * gs;
    const double gx = gxf;
    const long long io = (long long)o * npix + p;
    const double lo = L[io], t = (double)U[io] + lo / rho;
    dx[p] = (float)(aE * gx);
    sr += gx * ((1.0 - aE) * (-lo / (rho * rho)) - (double)e2 * eta2 * aE1 * ((double)x[p] - t));
    const float xsp = xs[p];
    const float cl = (float)((1.0 - aE) * gx / rho), cu = (float)((1.0 - aE) * gx);
    for (int k = 0; k < m; ++k) {
      const long long i = (long long)k * npix + p;
      const float g = GL[i];
      dL[i] = k == o ? g + cl : g;
      dU[i] = k == o ? rho_f * g + cu : rho_f * g;
      sr += (double)g * ((double)U[i] - (double)xsp);
    }
  }
  wg_sum3(sr, 0.0, 0.0, part);
}

// ---------------------------------------------------------------------------
// x-update, AVG
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(UT) void k_unroll_xavg(int m, long long npix, const float* U, const float* L,
                                                    const float* scal, float* xo) {
  const float rho = scal[0];
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    float s = 0.f;
    for (int k = 0; k < m; ++k) s += U[(long long)k * npix + p] + L[(long long)k * npix + p] / rho;
    xo[p] = s / (float)m;
  }
}

// dU_m = G / M, dL_m = G / (M rho), d rho = -sum_m sum G L_m / (M rho^2)
__global__ __launch_bounds__(UT) void k_unroll_xavg_grad(int m, long long npix, const float* G, const float* L,
                                                         const float* scal, float* dU, float* dL, double* part) {
  const double rho = scal[0];
  double sr = 0.0;
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    const double g = G[p];
    double sl = 0.0;
    for (int k = 0; k < m; ++k) {
      const long long i = (long long)k * npix + p;
      dU[i] = (float)(g / m);
      dL[i] = (float)(g / (m * rho));
      sl += L[i];
    }
    sr -= g * sl / (m * rho * rho);
  }
  wg_sum3(sr, 0.0, 0.0, part);
}

// ---------------------------------------------------------------------------
// dual update
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(UT) void k_unroll_dual(int m, long long npix, const float* L, const float* U,
                                                    const float* xn, const float* scal, float* Lo) {
  const float rho = scal[0];
  const long long total = (long long)m * npix;
  for (long long i = ((long long)blockIdx.x * UT + threadIdx.x); i < total; i += (long long)gridDim.x * UT)
    Lo[i] = L[i] + rho * (U[i] - xn[i % npix]);
}

// dL = G, dU = rho G, dx' = -rho sum_m G_m, d rho = sum G (U - x')
__global__ __launch_bounds__(UT) void k_unroll_dual_grad(int m, long long npix, const float* G, const float* U,
                                                         const float* xn, const float* scal, float* dL, float* dU,
                                                         float* dxn, double* part) {
  const float rho = scal[0];
  double sr = 0.0;
  for (long long p = (long long)blockIdx.x * UT + threadIdx.x; p < npix; p += (long long)gridDim.x * UT) {
    const float xp = xn[p];
    float gs = 0.f;
    for (int k = 0; k < m; ++k) {
      const long long i = (long long)k * npix + p;
      const float g = G[i];
      dL[i] = g;
      dU[i] = rho * g;
      gs += g;
      sr += (double)g * ((double)U[i] - (double)xp);
    }
    dxn[p] = -rho * gs;
  }
  wg_sum3(sr, 0.0, 0.0, part);
}

// out = alpha a + beta b (the residual P U - D of the unrolled u-step)
__global__ __launch_bounds__(UT) void k_axpby(long long n, float alpha, const float* a, float beta, const float* b,
                                              float* out) {
  for (long long i = (long long)blockIdx.x * UT + threadIdx.x; i < n; i += (long long)gridDim.x * UT)
    out[i] = alpha * a[i] + beta * b[i];
}

// ---------------------------------------------------------------------------
// finish: adds the partials in a fixed order (thread t takes partials t, t +
// UT, ...; then a fixed tree over the threads) and forms the scalar gradients
//   kind 0 (u-step):  parts A (<G, U - x>, <G, L>) over na workgroups, parts B
//                     (<P G, R>) over nb: d rho = -eta sux, d eta = -(sr + rho sux + sl)
//   kind 1 (one sum): d rho = sum of parts A, d eta = 0
// With acc the two values are added to dscal instead of written.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(UT) void k_unroll_finish(int kind, const double* pa, int na, const double* pb, int nb,
                                                      const float* scal, float* dscal, int acc) {
  __shared__ double red[3][UT];
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int i = t; i < na; i += UT) { a0 += pa[3 * i]; a1 += pa[3 * i + 1]; }
  for (int i = t; i < nb; i += UT) a2 += pb[3 * i];
  red[0][t] = a0; red[1][t] = a1; red[2][t] = a2;
  __syncthreads();
  for (int o = UT / 2; o > 0; o >>= 1) {
    if (t < o) {
      red[0][t] += red[0][t + o];
      red[1][t] += red[1][t + o];
      red[2][t] += red[2][t + o];
    }
    __syncthreads();
  }
  if (t != 0) return;
  const double s0 = red[0][0], s1 = red[1][0], s2 = red[2][0];
  float r0, r1;
  if (kind == 0) {
    const double rho = scal[0], eta = scal[1];
    r0 = (float)(-eta * s0);
    r1 = (float)(-(s2 + rho * s0 + s1));
  } else {
    r0 = (float)s0;
    r1 = 0.f;
  }
  dscal[0] = acc ? dscal[0] + r0 : r0;
  dscal[1] = acc ? dscal[1] + r1 : r1;
}

}  // namespace tomo
