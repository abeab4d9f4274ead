// Shared device-side definitions of the tomoadmm HIP library (gfx950): job
// sources and the projector / backprojector descriptors (the consensus,
// quantizer and regularization descriptors are in consensus.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tomo {

// ---------------------------------------------------------------------------
// Work descriptors.  A launch processes one descriptor passed by value
// (Single) or many descriptors in device memory (Many); a descriptor owns the
// contiguous range of workgroup ids [wg_begin, wg_begin + its WG count).
// ---------------------------------------------------------------------------
template <class Job>
struct Single {
  Job job;
  __device__ __forceinline__ Job get(int bid, int& lid) const {
    lid = bid;
    return job;
  }
};

template <class Job>
struct Many {
  const Job* jobs;
  int n_jobs;
  // optional dispatch order: workgroup b of the launch runs entry order[b] =
  // {job, workgroup within the job}; null runs the jobs in table order
  const int2* order = nullptr;
  __device__ __forceinline__ Job get(int bid, int& lid) const {
    if (order) {
      const int2 e = order[bid];
      lid = e.y;
      return jobs[e.x];
    }
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {  // last job with wg_begin <= bid (uniform across the WG)
      int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].wg_begin <= bid) lo = mid; else hi = mid - 1;
    }
    Job j = jobs[lo];
    lid = bid - j.wg_begin;
    return j;
  }
};

// ---------------------------------------------------------------------------
// Forward projector: one job = one image and one set of angles.
// Decomposition: angle chunks of PA angles x rectangular image regions.
// Each (chunk, region) workgroup writes partial ray sums; with more than one
// region a reduction launch (one workgroup per chunk) adds them in order.
// ---------------------------------------------------------------------------
constexpr int PA = 4;          // angles per workgroup
constexpr int PREG = 256;      // max region side
constexpr int PACC = 384;      // ray accumulators per angle and region (>= PREG * sqrt(2) + 3)
constexpr int PMAXREG = 256;   // max regions per job
constexpr int PTHREADS = 256;

// Region-resident projector: 128 x 128 regions held in LDS for all angles of
// a node; one workgroup per region, partials [n_ang][G][QACC].
constexpr int QR = 128;        // region side
constexpr int QOFF = 2;        // zero samples before each LDS line
constexpr int QLS = QR + 4;    // LDS line stride (zero samples on both sides)
constexpr int QACC = 192;      // rays per angle and region (>= 128 * sqrt(2) + 3)
constexpr int QBAND = 32;      // lines per unrolled band
constexpr int QTHREADS = 1024;
constexpr int QAG = 64;        // angles whose parameters are staged together
constexpr int QMAXN = QR * 16; // images up to this side (at most PMAXREG regions)

struct ProjJob {
  const float* img;     // [n][n]
  const double* ang;    // [n_ang]
  const float* d;       // [n_ang][nb] or null: out = scale * P img - d
  float* out;           // [n_ang][nb]
  float* partial;       // band kernel: [n_achunk][G][PA][PACC]; region-resident: [n_ang][G][QACC]
  int* bbase;           // band kernel, G > 1: [n_achunk][G][PA] first bin of each region's partials
  int n, nb, n_ang;
  int n_achunk;
  int reg_h, reg_w;     // region size (<= PREG)
  int n_rr, n_rc;       // regions down / across
  int wg_begin;         // first workgroup of this job in its launch
  float scale;
  int chord;            // 0: Joseph weights; 1: chord lengths (intersection lengths)
};

// ---------------------------------------------------------------------------
// Backprojector: one job = one image tile grid and one set of angles.
// ---------------------------------------------------------------------------
constexpr int BT = 32;          // tile side in pixels
constexpr int BW = 48;          // staged bins per (tile, angle)
constexpr int BAC = 64;         // angles per staged chunk
constexpr int BTHREADS = 256;   // 4 pixels per thread

enum { BP_PLAIN = 0, BP_ADMM = 1, BP_UNROLL = 2 };

struct BPJob {
  const float* sino;    // [n_ang][nb]
  const double* ang;    // [n_ang]
  float* img;           // output image (plain) or u (ADMM)
  const float* x;       // ADMM: consensus image
  const float* lam;     // ADMM: dual variable
  int n, nb, n_ang;
  int tiles_x;          // tiles per row
  int wg_begin;
  int mode;
  float alpha, beta;    // plain: img = alpha * P^T sino + beta * img
  float rho, eta1;      // ADMM:  u -= eta1 * (P^T sino + rho (u - x) + lam)
  int chord;            // 0: Joseph weights; 1: chord lengths
  const float* u_in;    // unrolled step: u read from here (img = the new u), or null (u = img)
  const float* scal;    // unrolled step: (rho, eta1) in device memory, or null (the fields above)
};

// cos and sin of a projection angle.  The chord-length model takes a cosine
// or sine within 1e-12 of zero as exactly zero (the angle is axis-aligned and
// lines on pixel edges follow the half-open pixel convention); the Joseph
// model uses the values as computed.
__host__ __device__ __forceinline__ void angle_trig(double th, int chord, double& cs, double& sn) {
  double c = cos(th), s = sin(th);
  if (chord) {
    const bool zc = fabs(c) < 1e-12, zs = fabs(s) < 1e-12;
    const double c1 = zs ? (c > 0.0 ? 1.0 : -1.0) : (zc ? 0.0 : c);
    const double s1 = zc ? (s > 0.0 ? 1.0 : -1.0) : (zs ? 0.0 : s);
    c = c1;
    s = s1;
  }
  cs = c;
  sn = s;
}

}  // namespace tomo
