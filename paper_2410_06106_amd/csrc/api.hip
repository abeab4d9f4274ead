// C ABI of the tomoadmm library: argument checks, workspace and plans, launches.
#include <algorithm>
#include <initializer_list>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "consensus.h"
#include "codec.h"
#include "../../include/tomoadmm.h"

namespace tomo {
template <int R, class Src, bool CHORD> __global__ void k_project(Src);
template <class Src> __global__ void k_project_reduce(Src);
template <class Src> __global__ void k_project_res(Src);
template <class Src> __global__ void k_project_res_reduce(Src);
template <class Src, bool CHORD> __global__ void k_backproject(Src);
__global__ void k_seg_none(const SegJob*, int, int);
template <bool REG, bool TZ> __global__ void k_kmeans(const KMJob*, KMJob, int, int, int, const KMBlock*);
__global__ void k_dct_range(const SegJob*, int, int, SegJob, int, int);
__global__ void k_dct_code(const SegJob*, int, int, SegJob, int);
__global__ void k_avg(Many<AvgJob>, const NodeRef*);
__global__ void k_dual(Many<NodeRef>);
__global__ void k_reg_step(Many<RegJob>, int);
__global__ void k_sqdiff(const float*, const float*, long long, double*);
__global__ void k_pack_labels(const uint8_t*, int, int, unsigned*, long long);
__global__ void k_ecode_bits(const int16_t*, int, int, int, unsigned*);
__global__ void k_ecode_scan(unsigned*, int, unsigned*, unsigned*);
__global__ void k_ecode_zero(unsigned*, long long);
__global__ void k_ecode_write(const int16_t*, int, int, int, const unsigned*, unsigned*);
__global__ void k_ecode_decode(const unsigned*, long long, const unsigned*, const unsigned*, int, int, int16_t*, int,
                               int*);
__global__ void k_unpack_labels(const unsigned*, int, int, const float*, int, uint8_t*, float*);
__global__ void k_unroll_ustep(int, long long, const float*, const float*, const float*, const float*, const float*,
                               float*);
__global__ void k_unroll_ustep_grad(int, long long, const float*, const float*, const float*, const float*,
                                    const float*, const float*, float*, float*, float*, int, double*);
__global__ void k_unroll_dot(long long, const float*, const float*, double*);
__global__ void k_unroll_xseg(int, const int*, const float*, const float*, const float*, const float*, float, int,
                              float*);
__global__ void k_unroll_xseg_grad(int, int, const int*, const float*, const float*, const float*, const float*,
                                   const float*, float, int, float*, float*, float*, double*);
__global__ void k_unroll_segdual_grad(int, int, const int*, const float*, const float*, const float*, const float*,
                                      const float*, const float*, const float*, float, int, float*, float*, float*,
                                      double*);
__global__ void k_unroll_xavg(int, long long, const float*, const float*, const float*, float*);
__global__ void k_unroll_xavg_grad(int, long long, const float*, const float*, const float*, float*, float*,
                                   double*);
__global__ void k_unroll_dual(int, long long, const float*, const float*, const float*, const float*, float*);
__global__ void k_unroll_dual_grad(int, long long, const float*, const float*, const float*, const float*, float*,
                                   float*, float*, double*);
__global__ void k_unroll_finish(int, const double*, int, const double*, int, const float*, float*, int);
__global__ void k_axpby(long long, float, const float*, float, const float*, float*);
}  // namespace tomo

using namespace tomo;

// Range partials of quantize_dct_noalloc: one array per device, held until the
// process ends and shared by every call on that device.  In host code its name
// is only a stand-in for the symbol: kernels get the device address that
// hipGetSymbolAddress returns, looked up once per device by tomo_create.
static __device__ __align__(256) float4 scratch[DCT_MAX_CHUNKS];

static_assert(sizeof(tomo_node) == 80, "tomo_node must have no padding (plans compare it bytewise)");
static_assert(sizeof(tomo_msg) == 48, "tomo_msg must have no padding");
static_assert(sizeof(tomo_proj_item) == 40, "tomo_proj_item must have no padding (plans compare it bytewise)");

namespace {

constexpr int kMaxRegions = PMAXREG;  // regions per projector job (finalizer table size)

// Device buffer that only grows.  A smaller allocation it replaces is kept
// until release() or destruction, so work captured into a graph earlier still
// finds its memory.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  std::vector<void*> old;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  bool ensure(size_t want) {
    if (want <= bytes) return true;
    void* q = nullptr;
    if (hipMalloc(&q, want) != hipSuccess) return false;
    if (p) old.push_back(p);
    p = q;
    bytes = want;
    return true;
  }
  void release() {
    for (void* q : old) (void)hipFree(q);
    old.clear();
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Pinned host staging for job tables uploaded on every call: a slot is reused
// only after the copy that read it has completed (an event per slot).
struct HostRing {
  static constexpr int kSlots = 4;
  void* host[kSlots] = {};
  size_t bytes[kSlots] = {};
  hipEvent_t ev[kSlots] = {};
  int next = 0;
  HostRing() = default;
  HostRing(const HostRing&) = delete;
  HostRing& operator=(const HostRing&) = delete;
  ~HostRing() {
    for (int i = 0; i < kSlots; ++i) {
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      if (host[i]) (void)hipHostFree(host[i]);
    }
  }
  // a slot of at least `want` bytes, or nullptr
  void* acquire(size_t want, int& slot) {
    slot = next;
    next = (next + 1) % kSlots;
    if (ev[slot] && hipEventSynchronize(ev[slot]) != hipSuccess) return nullptr;
    if (bytes[slot] < want) {
      if (host[slot]) (void)hipHostFree(host[slot]);
      host[slot] = nullptr;
      bytes[slot] = 0;
      if (hipHostMalloc(&host[slot], want) != hipSuccess) return nullptr;
      bytes[slot] = want;
    }
    return host[slot];
  }
  // after the copy out of `slot` has been enqueued on `stream`
  bool mark(int slot, hipStream_t stream) {
    if (!ev[slot] && hipEventCreateWithFlags(&ev[slot], hipEventDisableTiming) != hipSuccess) return false;
    return hipEventRecord(ev[slot], stream) == hipSuccess;
  }
};

// Projector decomposition of one job: angle chunks x regions.
struct ProjShape {
  int n_achunk, reg_h, reg_w, n_rr, n_rc;
  int wgs() const { return n_achunk * n_rr * n_rc; }
  int regions() const { return n_rr * n_rc; }
};

int reduce_wgs(const ProjShape& s, int n_bins) {
  return s.n_achunk * ((n_bins + PTHREADS - 1) / PTHREADS);
}

// Region-resident projector: one workgroup per 128 x 128 region of a node,
// every angle of the node in it.
ProjShape resident_shape(int n) {
  ProjShape s;
  s.n_achunk = 1;
  s.reg_h = s.reg_w = std::min(n, QR);
  s.n_rr = s.n_rc = (n + s.reg_h - 1) / s.reg_h;
  return s;
}

int resident_reduce_wgs(int n_ang, int n_bins) { return n_ang * ((n_bins + QTHREADS - 1) / QTHREADS); }

// Estimated run time of every workgroup of one band-projector job, appended to
// `cost` in the job's workgroup order, in units of one wave's pass of 64 rays
// through a band: per band of R driving lines, the rays of the band's angle
// class (the kernel's own ray range, affine in the band start) shared by the
// four waves, plus one unit for staging the band and one per workgroup.  Only
// the dispatch order depends on it, never a result.
void band_costs(const double* ang, int n_ang, int n, int nb, const ProjShape& s, int R, int chord,
                std::vector<float>& cost) {
  const double h = 0.5 * (n - 1), hb = 0.5 * (nb - 1);
  const int PAD = R + 4, per_round = 64 * (PTHREADS / 64);
  for (int ac = 0; ac < s.n_achunk; ++ac)
    for (int g = 0; g < s.regions(); ++g) {
      const int rr = g / s.n_rc, rc = g - rr * s.n_rc;
      const int gr0 = rr * s.reg_h, gc0 = rc * s.reg_w;
      const int gh = std::min(s.reg_h, n - gr0), gw = std::min(s.reg_w, n - gc0);
      const int na = std::min(PA, n_ang - ac * PA);
      int cls[PA], bb[PA];
      double lo[PA], hi[PA], sl[PA];
      for (int a = 0; a < na; ++a) {
        double cs, sn;
        angle_trig(ang[ac * PA + a], chord, cs, sn);
        const double s00 = (gc0 - h) * cs + (gr0 - h) * sn + hb;
        bb[a] = (int)std::floor(s00 + std::min(0.0, (gw - 1) * cs) + std::min(0.0, (gh - 1) * sn));
        const bool rows = std::fabs(cs) >= std::fabs(sn);
        const double ib = rows ? cs : sn, gam = rows ? -sn / cs : -cs / sn;
        const double xi0 = rows ? (bb[a] - hb - (gr0 - h) * sn) / cs + h - gc0 + PAD
                                : (bb[a] - hb - (gc0 - h) * cs) / sn + h - gr0 + PAD;
        const int W = rows ? gw : gh;
        const double span = (R - 1) * gam;
        const double t1 = (PAD - 1 - xi0 - std::max(0.0, span)) * ib;
        const double t2 = (PAD + W - xi0 - std::min(0.0, span)) * ib;
        cls[a] = rows ? 0 : 1;
        lo[a] = std::min(t1, t2);
        hi[a] = std::max(t1, t2);
        sl[a] = -gam * ib;
      }
      float c = 1.f;
      for (int k = 0; k < 2; ++k) {
        bool any = false;
        for (int a = 0; a < na; ++a) any |= cls[a] == k;
        if (!any) continue;
        const int D = k == 0 ? gh : gw;
        for (int db = 0; db < D; db += R) {
          int tot = 0;
          for (int a = 0; a < na; ++a) {
            if (cls[a] != k) continue;
            const int jl = std::max((int)std::floor(lo[a] + db * sl[a]), std::max(0, -bb[a]));
            const int jh = std::min((int)std::ceil(hi[a] + db * sl[a]), std::min(PACC - 1, nb - 1 - bb[a]));
            tot += std::max(0, jh - jl + 1);
          }
          c += 1.f + (float)((tot + per_round - 1) / per_round);
        }
      }
      cost.push_back(c);
    }
}

constexpr int kOrderMaxWgsPerCu = 8;   // largest launch (workgroups per CU) given a dispatch order

// Dispatch order of a batched band-projector launch.  Workgroups are dealt to
// the dies round-robin (workgroup b runs on die b % n_xcc, each die with its
// own L2), and the workgroups resident on one die's compute units share them.
// So: (1) the workgroups of one (job, region) pair form a group that reads one
// region of one image; the groups go to the dies heaviest first (estimated
// cost), each into the least loaded die with room left (a die holds its share
// of the launch's workgroups; a group that does not fit continues in the next
// such die), so that each region is read on about one die and the dies finish
// together; (2) each die's list is sorted by cost, largest first (ties keep
// table order), so that a compute unit receives a mix of heavy and light
// workgroups and the longest ones do not trail at the end; (3) the lists are
// interleaved: blockIdx b takes entry b / n_xcc of the list of die b % n_xcc.
// With `per_node` the groups are whole jobs (every region and angle chunk of
// a node), and job_die receives the die each job starts on, so that the
// region reduction and the backprojection of that node can run there too.
// Needs the angles on the host; returns false (and the launch keeps table
// order) when they cannot be read.
bool band_order(const tomo_node* nodes, int n_nodes, const std::vector<ProjShape>& shapes,
                const std::vector<ProjJob>& pj, int R, int chord, int n_xcc, bool per_node,
                std::vector<int2>& order, std::vector<int>& job_die) {
  std::vector<float> cost;
  std::vector<int2> ent;
  std::vector<std::vector<int>> groups;
  std::vector<double> gcost;
  std::vector<double> ang;
  for (int i = 0; i < n_nodes; ++i) {
    ang.resize(nodes[i].n_ang);
    if (hipMemcpy(ang.data(), nodes[i].angles, ang.size() * sizeof(double), hipMemcpyDefault) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    const int c0 = (int)cost.size();
    if (pj[i].wg_begin != c0) return false;
    band_costs(ang.data(), nodes[i].n_ang, nodes[i].g.n, nodes[i].g.n_bins, shapes[i], R, chord, cost);
    for (int k = c0; k < (int)cost.size(); ++k) ent.push_back(make_int2(i, k - c0));
    const int G = shapes[i].regions();
    if (per_node) {
      groups.emplace_back();
      double sum = 0.0;
      for (int k = c0; k < (int)cost.size(); ++k) {
        groups.back().push_back(k);
        sum += cost[k];
      }
      gcost.push_back(sum);
      continue;
    }
    for (int g = 0; g < G; ++g) {
      groups.emplace_back();
      double sum = 0.0;
      for (int ac = 0; ac < shapes[i].n_achunk; ++ac) {
        groups.back().push_back(c0 + ac * G + g);
        sum += cost[c0 + ac * G + g];
      }
      gcost.push_back(sum);
    }
  }
  const int T = (int)cost.size(), nx = std::max(1, std::min(n_xcc, T));
  std::vector<int> gi(groups.size());
  for (size_t k = 0; k < gi.size(); ++k) gi[k] = (int)k;
  std::stable_sort(gi.begin(), gi.end(), [&](int a, int b) { return gcost[a] > gcost[b]; });
  std::vector<std::vector<int>> die(nx);
  std::vector<double> load(nx, 0.0);
  std::vector<int> room(nx);
  for (int x = 0; x < nx; ++x) room[x] = T / nx + (x < T % nx ? 1 : 0);   // workgroups b with b % nx == x
  job_die.assign(n_nodes, -1);
  for (int g : gi) {
    size_t k = 0;
    while (k < groups[g].size()) {
      int best = -1;
      for (int x = 0; x < nx; ++x)
        if (room[x] > 0 && (best < 0 || load[x] < load[best])) best = x;
      if (best < 0) return false;
      const int job = ent[groups[g][k]].x;
      if (job_die[job] < 0) job_die[job] = best;
      for (; k < groups[g].size() && room[best] > 0; ++k) {
        die[best].push_back(groups[g][k]);
        load[best] += cost[groups[g][k]];
        --room[best];
      }
    }
  }
  order.resize(T);
  for (int x = 0; x < nx; ++x) {
    std::stable_sort(die[x].begin(), die[x].end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (size_t k = 0; k < die[x].size(); ++k) order[k * nx + x] = ent[die[x][k]];
  }
  return true;
}

// Dispatch order that runs the workgroups of job i (wgs[i] of them, in job
// order) on die job_die[i]: each die's list interleaved as in band_order.
// Only when every die receives the same number of workgroups (a launch has no
// holes); returns false otherwise, and the launch keeps table order.
bool die_order(const std::vector<int>& wgs, const std::vector<int>& job_die, int n_xcc, std::vector<int2>& order) {
  const int nx = std::max(1, n_xcc);
  std::vector<std::vector<int2>> die(nx);
  for (size_t i = 0; i < wgs.size(); ++i) {
    if (job_die[i] < 0 || job_die[i] >= nx) return false;
    for (int w = 0; w < wgs[i]; ++w) die[job_die[i]].push_back(make_int2((int)i, w));
  }
  for (int x = 1; x < nx; ++x)
    if (die[x].size() != die[0].size()) return false;
  order.resize(die[0].size() * nx);
  for (int x = 0; x < nx; ++x)
    for (size_t k = 0; k < die[x].size(); ++k) order[k * nx + x] = die[x][k];
  return true;
}

ProjShape base_shape(int n, int n_ang) {
  ProjShape s;
  s.n_achunk = (n_ang + PA - 1) / PA;
  s.reg_h = s.reg_w = std::min(n, PREG);
  s.n_rr = s.n_rc = (n + s.reg_h - 1) / s.reg_h;
  return s;
}

// Halve the regions of a job (rows first, sides >= 64) until the job alone
// spans kJobWGs workgroups.  The decomposition depends on the job only, so a
// node gives bit-identical results whether it is launched alone or batched.
// Region sides stay multiples of 16 so that rows of a region start on
// 16-byte boundaries whenever the image side is a multiple of 4.
void split_for_parallelism(ProjShape& s, int n, int job_wgs) {
  auto half = [](int r) { return ((r / 2) + 15) & ~15; };
  while (s.wgs() < job_wgs) {
    ProjShape c = s;
    if (c.reg_h >= c.reg_w && c.reg_h >= 128) {
      c.reg_h = half(c.reg_h); c.n_rr = (n + c.reg_h - 1) / c.reg_h;
    } else if (c.reg_w >= 128) {
      c.reg_w = half(c.reg_w); c.n_rc = (n + c.reg_w - 1) / c.reg_w;
    } else {
      break;
    }
    if (c.regions() > kMaxRegions) break;
    s = c;
  }
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

struct LocalPlan {
  std::vector<tomo_node> key;
  DevBuf pjobs, rjobs, bjobs, resid, partial, bbase;
  DevBuf order;                  // band projector dispatch order (int2 per workgroup), if built
  bool ordered = false;
  DevBuf rorder, border;         // reduction and backprojector orders (same die per node), if built
  bool r_ordered = false, b_ordered = false;
  int n_p = 0, p_wgs = 0, n_r = 0, r_wgs = 0, n_b = 0, b_wgs = 0;
  int band = 16;                 // projector band depth (16 or 32)
  bool resident = false;         // region-resident projector (k_project_res)
  bool chord = false;            // chord-length model
};

struct ConsPlan {
  std::vector<tomo_node> key;
  std::vector<tomo_msg> msg_key;
  std::vector<tomo_reg> reg_key;
  DevBuf seg, avg, noderefs, kmjobs, kmwork, kmblocks, dctpart;
  int dct_range_wgs = 0, dct_code_wgs = 0;   // DCT codec launches
  int dct_range_uni = 0, dct_code_uni = 0;   // workgroups of every job, when all jobs have the same (else 0)
  int n_seg = 0, n_avg = 0, avg_wgs = 0, dual_wgs = 0;
  bool any_xt = false;   // some message asks for the segment before Q
  int n_refs = 0;                 // dual-update entries: the nodes, then the regularization blocks
  int km_small = 0, km_big = 0;   // K-means jobs regrouping in LDS, then those using the workspace
};

constexpr int kKmThreads = 1024;

// z-update of a list of regularization blocks: job table and the TV blocks'
// scratch fields, built once per block array (and the slices' images)
struct RegPlan {
  std::vector<tomo_reg> key;
  std::vector<const float*> xs;   // each block's slice image and side: part of the key
  std::vector<int> ns;
  DevBuf jobs, scratch;
  int n_jobs = 0, wgs = 0;
  int launches = 1;               // k_reg_step launches of one z-update (the most any block needs)
};

// FNV-1a hash of a descriptor array: the plan caches are indexed by it.
uint64_t hash_bytes(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

bool same_nodes(const std::vector<tomo_node>& k, const tomo_node* nodes, int n) {
  return (int)k.size() == n && std::memcmp(k.data(), nodes, sizeof(tomo_node) * n) == 0;
}

}  // namespace

struct tomo_ctx {
  int device = 0;
  int n_cu = 1;
  int n_xcc = 1;              // accelerator complex dies: workgroup b of a launch runs on die b % n_xcc
  int proj_job_wgs = 16;      // TOMO_OPT_PROJ_JOB_WGS
  int proj_band = 32;         // TOMO_OPT_PROJ_BAND
  int proj_kernel = 0;        // TOMO_OPT_PROJ_KERNEL
  int model = 0;              // TOMO_OPT_PROJ_MODEL (0 Joseph, 1 chord lengths)
  int proj_order = 2;         // TOMO_OPT_PROJ_ORDER (0 table order, 1 estimated cost, largest first,
                              // 2 the same with each node's workgroups of every local-update kernel on one die)
  std::string err;
  DevBuf partial;                                // standalone projector workspace
  DevBuf pbbase;                                 // standalone projector: region bin bases
  DevBuf km_work;                                // standalone K-means workspace
  DevBuf dct_part;                               // standalone DCT codec: range partials
  DevBuf unroll_part;                            // unrolled form: float64 partial sums
  DevBuf ctr_resid;                              // residual of tomo_ctr_gd
  DevBuf ecode_off;                              // block offsets of tomo_dct_encode
  std::vector<std::unique_ptr<LocalPlan>> lplans;
  std::vector<std::unique_ptr<ConsPlan>> cplans;
  std::unordered_multimap<uint64_t, LocalPlan*> lindex;   // hash of the node array -> plan
  std::unordered_multimap<uint64_t, ConsPlan*> cindex;    // hash of nodes and messages -> plan
  // plans dropped by tomo_set_option stay allocated (a captured graph may
  // still reference their buffers) until the context is destroyed
  std::vector<std::unique_ptr<LocalPlan>> retired_l;
  std::vector<std::unique_ptr<ConsPlan>> retired_c;
  std::vector<std::unique_ptr<RegPlan>> rplans;   // z-update plans (independent of the options)
  // tomo_project_many / tomo_backproject_many: job tables staged per call
  HostRing ring;
  DevBuf btable, bpartial, bbbase;
  int fail(int code, const std::string& msg) { err = msg; return code; }
};

namespace {

int launch_status(tomo_ctx* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx->fail(TOMO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return TOMO_OK;
}

int set_device(tomo_ctx* ctx) {
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(TOMO_EDEVICE, "hipSetDevice failed");
  return TOMO_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float4* g_scratch_ptr[kMaxDevices] = {};

// With the device current: the device address of its scratch array (once).
int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return TOMO_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return TOMO_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TOMO_EDEVICE;
  g_scratch_ptr[device] = static_cast<float4*>(p);
  return TOMO_OK;
}

float4* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

int check_geom(tomo_ctx* ctx, tomo_geom g) {
  if (g.n < 1 || g.n_bins < 1) return ctx->fail(TOMO_EINVAL, "geometry needs n >= 1 and n_bins >= 1");
  // the projector's finalizer holds at most PMAXREG regions of <= PREG x PREG pixels
  if (g.n > 16 * PREG || (long long)g.n_bins > (1 << 24))
    return ctx->fail(TOMO_EUNSUPPORTED, "image side above 4096 or more than 2^24 bins");
  return TOMO_OK;
}

ProjJob make_proj_job(const float* img, const double* ang, const float* d, float* out, int n, int nb,
                      int n_ang, const ProjShape& s) {
  ProjJob j{};
  j.img = img; j.ang = ang; j.d = d; j.out = out;
  j.n = n; j.nb = nb; j.n_ang = n_ang;
  j.n_achunk = s.n_achunk;
  j.reg_h = s.reg_h; j.reg_w = s.reg_w; j.n_rr = s.n_rr; j.n_rc = s.n_rc;
  j.scale = 1.f;
  return j;
}

BPJob make_bp_job(const float* sino, const double* ang, float* img, int n, int nb, int n_ang) {
  BPJob j{};
  j.sino = sino; j.ang = ang; j.img = img;
  j.n = n; j.nb = nb; j.n_ang = n_ang;
  j.tiles_x = (n + BT - 1) / BT;
  return j;
}

int check_nodes(tomo_ctx* ctx, const tomo_node* nodes, int n_nodes) {
  if (!nodes || n_nodes < 1) return ctx->fail(TOMO_EINVAL, "empty node list");
  for (int i = 0; i < n_nodes; ++i) {
    const tomo_node& N = nodes[i];
    if (int rc = check_geom(ctx, N.g)) return rc;
    if (N.n_ang < 1) return ctx->fail(TOMO_EINVAL, "node without angles");
    if (!N.angles || !N.d || !N.u || !N.lam || !N.x) return ctx->fail(TOMO_EINVAL, "null node pointer");
    if (N.seg_row0 < 0 || N.seg_rows < 1 || N.seg_row0 + N.seg_rows > N.g.n)
      return ctx->fail(TOMO_EINVAL, "segment outside the image");
    if (!(N.rho > 0.f)) return ctx->fail(TOMO_EINVAL, "rho must be positive");
    size_t img = (size_t)N.g.n * N.g.n * sizeof(float);
    if (overlaps(N.u, img, N.lam, img) || overlaps(N.u, img, N.x, img) || overlaps(N.lam, img, N.x, img))
      return ctx->fail(TOMO_EINVAL, "u, lambda and x must not overlap");
    if (i > 0 && nodes[i - 1].slice == N.slice) {
      if (nodes[i - 1].x != N.x || nodes[i - 1].g.n != N.g.n)
        return ctx->fail(TOMO_EINVAL, "nodes of one slice must share x and n");
    }
  }
  std::vector<int32_t> starts;   // first slice id of every run of equal ids
  for (int i = 0; i < n_nodes; ++i)
    if (i == 0 || nodes[i - 1].slice != nodes[i].slice) starts.push_back(nodes[i].slice);
  std::sort(starts.begin(), starts.end());
  if (std::adjacent_find(starts.begin(), starts.end()) != starts.end())
    return ctx->fail(TOMO_EINVAL, "nodes of one slice must be adjacent");
  // The consensus kernels of different nodes write their segments of x at the
  // same time: the segments of a slice must be disjoint and the x arrays of
  // different slices must not overlap.
  std::vector<std::pair<int32_t, int32_t>> segs;   // (row0, rows) of one slice
  std::vector<std::pair<uintptr_t, size_t>> xs;    // (address, bytes) per slice
  for (int a = 0; a < n_nodes;) {
    int b = a;
    segs.clear();
    while (b < n_nodes && nodes[b].slice == nodes[a].slice) {
      segs.emplace_back(nodes[b].seg_row0, nodes[b].seg_rows);
      ++b;
    }
    std::sort(segs.begin(), segs.end());
    for (size_t j = 1; j < segs.size(); ++j)
      if (segs[j - 1].first + segs[j - 1].second > segs[j].first)
        return ctx->fail(TOMO_EINVAL, "segments of one slice overlap");
    xs.emplace_back(reinterpret_cast<uintptr_t>(nodes[a].x), (size_t)nodes[a].g.n * nodes[a].g.n * sizeof(float));
    a = b;
  }
  std::sort(xs.begin(), xs.end());
  for (size_t j = 1; j < xs.size(); ++j)
    if (xs[j - 1].first + xs[j - 1].second > xs[j].first)
      return ctx->fail(TOMO_EINVAL, "x of different slices overlap");
  return TOMO_OK;
}

LocalPlan* find_local_plan(tomo_ctx* ctx, const tomo_node* nodes, int n_nodes) {
  auto range = ctx->lindex.equal_range(hash_bytes(nodes, sizeof(tomo_node) * n_nodes));
  for (auto it = range.first; it != range.second; ++it)
    if (same_nodes(it->second->key, nodes, n_nodes)) return it->second;
  return nullptr;
}

uint64_t cons_hash(const tomo_node* nodes, int n_nodes, const tomo_msg* msg) {
  uint64_t h = hash_bytes(nodes, sizeof(tomo_node) * n_nodes);
  return msg ? hash_bytes(msg, sizeof(tomo_msg) * n_nodes, h) : h;
}

LocalPlan* get_local_plan(tomo_ctx* ctx, const tomo_node* nodes, int n_nodes, int& rc) {
  rc = TOMO_OK;
  if (LocalPlan* p = find_local_plan(ctx, nodes, n_nodes)) return p;
  auto plan = std::make_unique<LocalPlan>();
  plan->key.assign(nodes, nodes + n_nodes);
  std::vector<ProjShape> shapes;
  size_t resid_elems = 0, part_elems = 0;
  bool resident = ctx->proj_kernel == 1 && ctx->model == 0;
  for (int i = 0; i < n_nodes; ++i) resident = resident && nodes[i].g.n <= QMAXN;
  for (int i = 0; i < n_nodes; ++i) {
    if (resident) {
      shapes.push_back(resident_shape(nodes[i].g.n));
    } else {
      shapes.push_back(base_shape(nodes[i].g.n, nodes[i].n_ang));
      split_for_parallelism(shapes.back(), nodes[i].g.n, ctx->proj_job_wgs);
    }
  }
  std::vector<size_t> roff(n_nodes), poff(n_nodes), boff(n_nodes);
  size_t bb_elems = 0;
  for (int i = 0; i < n_nodes; ++i) {
    roff[i] = resid_elems;
    resid_elems += (size_t)nodes[i].n_ang * nodes[i].g.n_bins;
    poff[i] = part_elems;
    boff[i] = bb_elems;
    if (resident) {
      part_elems += (size_t)nodes[i].n_ang * shapes[i].regions() * QACC;
    } else if (shapes[i].regions() > 1) {
      part_elems += (size_t)shapes[i].wgs() * PA * PACC;
      bb_elems += (size_t)shapes[i].wgs() * PA;
    }
  }
  if (!plan->resid.ensure(resid_elems * 4) || !plan->partial.ensure(std::max<size_t>(part_elems, 1) * 4) ||
      !plan->bbase.ensure(std::max<size_t>(bb_elems, 1) * 4)) {
    rc = ctx->fail(TOMO_ENOMEM, "plan workspace allocation failed");
    return nullptr;
  }
  std::vector<ProjJob> pj, rj;
  std::vector<BPJob> bj;
  int pw = 0, rw = 0, bw = 0;
  float* R = static_cast<float*>(plan->resid.p);
  float* PP = static_cast<float*>(plan->partial.p);
  for (int i = 0; i < n_nodes; ++i) {
    const tomo_node& N = nodes[i];
    ProjJob j = make_proj_job(N.u, N.angles, N.d, R + roff[i], N.g.n, N.g.n_bins, N.n_ang, shapes[i]);
    j.chord = ctx->model;
    j.partial = PP + poff[i];
    j.bbase = static_cast<int*>(plan->bbase.p) + boff[i];
    j.wg_begin = pw;
    pw += shapes[i].wgs();
    pj.push_back(j);
    if (resident || shapes[i].regions() > 1) {     // reduction launch
      ProjJob r = j;
      r.wg_begin = rw;
      rw += resident ? resident_reduce_wgs(N.n_ang, N.g.n_bins) : reduce_wgs(shapes[i], N.g.n_bins);
      rj.push_back(r);
    }
    BPJob b = make_bp_job(R + roff[i], N.angles, N.u, N.g.n, N.g.n_bins, N.n_ang);
    b.mode = BP_ADMM;
    b.chord = ctx->model;
    b.x = N.x;
    b.lam = N.lam;
    b.rho = N.rho;
    b.eta1 = N.eta1;
    b.wg_begin = bw;
    bw += b.tiles_x * b.tiles_x;
    bj.push_back(b);
  }
  if (!plan->pjobs.ensure(pj.size() * sizeof(ProjJob)) || !plan->bjobs.ensure(bj.size() * sizeof(BPJob)) ||
      !plan->rjobs.ensure(std::max<size_t>(rj.size(), 1) * sizeof(ProjJob))) {
    rc = ctx->fail(TOMO_ENOMEM, "plan descriptor allocation failed");
    return nullptr;
  }
  if (hipMemcpy(plan->pjobs.p, pj.data(), pj.size() * sizeof(ProjJob), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(plan->bjobs.p, bj.data(), bj.size() * sizeof(BPJob), hipMemcpyHostToDevice) != hipSuccess ||
      (!rj.empty() &&
       hipMemcpy(plan->rjobs.p, rj.data(), rj.size() * sizeof(ProjJob), hipMemcpyHostToDevice) != hipSuccess)) {
    rc = ctx->fail(TOMO_EDEVICE, "descriptor upload failed");
    return nullptr;
  }
  std::vector<int2> ord;
  std::vector<int> job_die;
  auto upload = [&](DevBuf& buf, const std::vector<int2>& o) {
    return buf.ensure(o.size() * sizeof(int2)) &&
           hipMemcpy(buf.p, o.data(), o.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess;
  };
  // with many workgroups per CU the hardware's dynamic dispatch evens out the
  // load and table order keeps the angle chunks of one region together in
  // time (shared reads in L2); the table pays off for launches of a few waves
  if (!resident && ctx->proj_order >= 1 && pw <= kOrderMaxWgsPerCu * ctx->n_cu &&
      band_order(nodes, n_nodes, shapes, pj, ctx->proj_band, ctx->model, ctx->n_xcc, ctx->proj_order == 2, ord,
                 job_die) &&
      (int)ord.size() == pw) {
    if (!upload(plan->order, ord)) {
      rc = ctx->fail(TOMO_EDEVICE, "dispatch order upload failed");
      return nullptr;
    }
    plan->ordered = true;
    if (ctx->proj_order == 2) {
      // each die reads only its own nodes' partials, residuals and images:
      // a node's reduction and backprojection workgroups run on its die too
      std::vector<int> rwgs, rdie, bwgs;
      for (int i = 0; i < n_nodes; ++i) {
        if (shapes[i].regions() > 1) {
          rwgs.push_back(reduce_wgs(shapes[i], nodes[i].g.n_bins));
          rdie.push_back(job_die[i]);
        }
        bwgs.push_back(bj[i].tiles_x * bj[i].tiles_x);
      }
      std::vector<int2> ro, bo;
      if (!rj.empty() && die_order(rwgs, rdie, ctx->n_xcc, ro) && (int)ro.size() == rw) {
        if (!upload(plan->rorder, ro)) {
          rc = ctx->fail(TOMO_EDEVICE, "dispatch order upload failed");
          return nullptr;
        }
        plan->r_ordered = true;
      }
      if (die_order(bwgs, job_die, ctx->n_xcc, bo) && (int)bo.size() == bw) {
        if (!upload(plan->border, bo)) {
          rc = ctx->fail(TOMO_EDEVICE, "dispatch order upload failed");
          return nullptr;
        }
        plan->b_ordered = true;
      }
    }
  }
  plan->n_r = (int)rj.size();
  plan->r_wgs = rw;
  plan->n_p = (int)pj.size();
  plan->p_wgs = pw;
  plan->n_b = (int)bj.size();
  plan->b_wgs = bw;
  plan->band = ctx->proj_band;
  plan->resident = resident;
  plan->chord = ctx->model == 1;
  ctx->lindex.emplace(hash_bytes(nodes, sizeof(tomo_node) * n_nodes), plan.get());
  ctx->lplans.push_back(std::move(plan));
  return ctx->lplans.back().get();
}

// Residual r = P u - d of every node of a plan: the region pass, then (for
// nodes split into several regions) the reduction pass.
// What one batched projection launch needs: the job tables on the device, the
// workgroup counts and the kernel choice.
struct ProjLaunch {
  const ProjJob* pjobs = nullptr;
  const ProjJob* rjobs = nullptr;
  const int2* order = nullptr;   // band kernel dispatch order or null
  const int2* rorder = nullptr;  // reduction dispatch order or null
  int n_p = 0, p_wgs = 0, n_r = 0, r_wgs = 0;
  int band = 32;
  bool resident = false, chord = false;
};

ProjLaunch launch_of(const LocalPlan* plan) {
  ProjLaunch L;
  L.pjobs = static_cast<const ProjJob*>(plan->pjobs.p);
  L.rjobs = static_cast<const ProjJob*>(plan->rjobs.p);
  L.order = plan->ordered ? static_cast<const int2*>(plan->order.p) : nullptr;
  L.rorder = plan->r_ordered ? static_cast<const int2*>(plan->rorder.p) : nullptr;
  L.n_p = plan->n_p;
  L.p_wgs = plan->p_wgs;
  L.n_r = plan->n_r;
  L.r_wgs = plan->r_wgs;
  L.band = plan->band;
  L.resident = plan->resident;
  L.chord = plan->chord;
  return L;
}

void launch_projection(const ProjLaunch& L, void* stream) {
  Many<ProjJob> ps{L.pjobs, L.n_p};
  if (L.resident) {
    Many<ProjJob> rs{L.rjobs, L.n_r};
    hipLaunchKernelGGL(k_project_res<Many<ProjJob>>, dim3(L.p_wgs), dim3(QTHREADS), 0, (hipStream_t)stream, ps);
    hipLaunchKernelGGL(k_project_res_reduce<Many<ProjJob>>, dim3(L.r_wgs), dim3(QTHREADS), 0, (hipStream_t)stream,
                       rs);
    return;
  }
  const dim3 grid(L.p_wgs), block(PTHREADS);
  ps.order = L.order;
  if (L.chord) {
    if (L.band == 32)
      hipLaunchKernelGGL((k_project<32, Many<ProjJob>, true>), grid, block, 0, (hipStream_t)stream, ps);
    else
      hipLaunchKernelGGL((k_project<16, Many<ProjJob>, true>), grid, block, 0, (hipStream_t)stream, ps);
  } else {
    if (L.band == 32)
      hipLaunchKernelGGL((k_project<32, Many<ProjJob>, false>), grid, block, 0, (hipStream_t)stream, ps);
    else
      hipLaunchKernelGGL((k_project<16, Many<ProjJob>, false>), grid, block, 0, (hipStream_t)stream, ps);
  }
  if (L.n_r > 0) {
    Many<ProjJob> rs{L.rjobs, L.n_r};
    rs.order = L.rorder;
    hipLaunchKernelGGL(k_project_reduce<Many<ProjJob>>, dim3(L.r_wgs), dim3(PTHREADS), 0, (hipStream_t)stream, rs);
  }
}

// The backprojector instantiation for the model (chord lengths or Joseph).
template <class Src>
void launch_backproject(Src src, int wgs, int chord, void* stream) {
  if (chord)
    hipLaunchKernelGGL((k_backproject<Src, true>), dim3(wgs), dim3(BTHREADS), 0, (hipStream_t)stream, src);
  else
    hipLaunchKernelGGL((k_backproject<Src, false>), dim3(wgs), dim3(BTHREADS), 0, (hipStream_t)stream, src);
}

// out = P img (- d when d is not null) for one job, on the context's
// standalone workspace: the projector the options select, then the region
// reduction when the image is split.  Arguments are checked by the caller.
int project_one(tomo_ctx* ctx, tomo_geom g, const double* angles, int n_ang, const float* img,
                const float* d, float* out, void* stream) {
  if (ctx->proj_kernel == 1 && ctx->model == 0 && g.n <= QMAXN) {
    const ProjShape rs = resident_shape(g.n);
    ProjJob j = make_proj_job(img, angles, d, out, g.n, g.n_bins, n_ang, rs);
    if (!ctx->partial.ensure((size_t)n_ang * rs.regions() * QACC * 4)) return ctx->fail(TOMO_ENOMEM, "workspace");
    j.partial = static_cast<float*>(ctx->partial.p);
    hipLaunchKernelGGL(k_project_res<Single<ProjJob>>, dim3(rs.regions()), dim3(QTHREADS), 0, (hipStream_t)stream,
                       Single<ProjJob>{j});
    hipLaunchKernelGGL(k_project_res_reduce<Single<ProjJob>>, dim3(resident_reduce_wgs(n_ang, g.n_bins)),
                       dim3(QTHREADS), 0, (hipStream_t)stream, Single<ProjJob>{j});
    return TOMO_OK;
  }
  ProjShape sh = base_shape(g.n, n_ang);
  split_for_parallelism(sh, g.n, ctx->proj_job_wgs);
  ProjJob j = make_proj_job(img, angles, d, out, g.n, g.n_bins, n_ang, sh);
  if (sh.regions() > 1) {
    if (!ctx->partial.ensure((size_t)sh.wgs() * PA * PACC * 4) || !ctx->pbbase.ensure((size_t)sh.wgs() * PA * 4))
      return ctx->fail(TOMO_ENOMEM, "workspace");
    j.partial = static_cast<float*>(ctx->partial.p);
    j.bbase = static_cast<int*>(ctx->pbbase.p);
  }
  j.chord = ctx->model;
  const dim3 grid(sh.wgs()), block(PTHREADS);
  const Single<ProjJob> src{j};
  if (ctx->model == 1) {
    if (ctx->proj_band == 32)
      hipLaunchKernelGGL((k_project<32, Single<ProjJob>, true>), grid, block, 0, (hipStream_t)stream, src);
    else
      hipLaunchKernelGGL((k_project<16, Single<ProjJob>, true>), grid, block, 0, (hipStream_t)stream, src);
  } else {
    if (ctx->proj_band == 32)
      hipLaunchKernelGGL((k_project<32, Single<ProjJob>, false>), grid, block, 0, (hipStream_t)stream, src);
    else
      hipLaunchKernelGGL((k_project<16, Single<ProjJob>, false>), grid, block, 0, (hipStream_t)stream, src);
  }
  if (sh.regions() > 1)
    hipLaunchKernelGGL(k_project_reduce<Single<ProjJob>>, dim3(reduce_wgs(sh, g.n_bins)), dim3(PTHREADS), 0,
                       (hipStream_t)stream, Single<ProjJob>{j});
  return TOMO_OK;
}

// Job tables of a batch of independent projections (kind 0: sino = P image)
// or backprojections (kind 1: image = alpha P^T sino + beta image), built on
// the host for this call, staged through pinned memory and copied to the
// device on `stream`; the projector's workspace is the context's.  No cache:
// the item pointers may differ on every call.
// The unrolled u-step's extra operands (tomo_unroll_local_step): the
// projector subtracts D's rows, the backprojector forms Uo_i in its epilogue.
struct UnrollArgs {
  const float* D;
  const float* x;
  const float* L;
  const float* scal;
  float* Uo;
};

int stage_batch(tomo_ctx* ctx, const tomo_proj_item* items, int n_items, int kind, float alpha, float beta,
                void* stream, ProjLaunch& plan, int& bp_wgs, const UnrollArgs* ua = nullptr) {
  std::vector<ProjJob> pj, rj;
  std::vector<BPJob> bj;
  if (kind == 0) {
    bool resident = ctx->proj_kernel == 1 && ctx->model == 0;
    for (int i = 0; i < n_items; ++i) resident = resident && items[i].g.n <= QMAXN;
    std::vector<ProjShape> shapes;
    size_t part_elems = 0, bb_elems = 0;
    std::vector<size_t> poff(n_items), boff(n_items);
    for (int i = 0; i < n_items; ++i) {
      if (resident) {
        shapes.push_back(resident_shape(items[i].g.n));
      } else {
        shapes.push_back(base_shape(items[i].g.n, items[i].n_ang));
        split_for_parallelism(shapes.back(), items[i].g.n, ctx->proj_job_wgs);
      }
      poff[i] = part_elems;
      boff[i] = bb_elems;
      if (resident) {
        part_elems += (size_t)items[i].n_ang * shapes[i].regions() * QACC;
      } else if (shapes[i].regions() > 1) {
        part_elems += (size_t)shapes[i].wgs() * PA * PACC;
        bb_elems += (size_t)shapes[i].wgs() * PA;
      }
    }
    if (!ctx->bpartial.ensure(std::max<size_t>(part_elems, 1) * 4) ||
        !ctx->bbbase.ensure(std::max<size_t>(bb_elems, 1) * 4))
      return ctx->fail(TOMO_ENOMEM, "batch workspace allocation failed");
    int pw = 0, rw = 0;
    size_t drow = 0;
    for (int i = 0; i < n_items; ++i) {
      const tomo_proj_item& I = items[i];
      const float* d = ua ? ua->D + drow * I.g.n_bins : nullptr;
      drow += I.n_ang;
      ProjJob j = make_proj_job(I.image, I.angles, d, I.sino, I.g.n, I.g.n_bins, I.n_ang, shapes[i]);
      j.partial = static_cast<float*>(ctx->bpartial.p) + poff[i];
      j.bbase = static_cast<int*>(ctx->bbbase.p) + boff[i];
      j.chord = ctx->model;
      j.wg_begin = pw;
      pw += shapes[i].wgs();
      pj.push_back(j);
      if (resident || shapes[i].regions() > 1) {
        ProjJob r = j;
        r.wg_begin = rw;
        rw += resident ? resident_reduce_wgs(I.n_ang, I.g.n_bins) : reduce_wgs(shapes[i], I.g.n_bins);
        rj.push_back(r);
      }
    }
    plan.n_p = (int)pj.size();
    plan.p_wgs = pw;
    plan.n_r = (int)rj.size();
    plan.r_wgs = rw;
    plan.resident = resident;
  } else {
    int bw = 0;
    for (int i = 0; i < n_items; ++i) {
      const tomo_proj_item& I = items[i];
      BPJob b = make_bp_job(I.sino, I.angles, I.image, I.g.n, I.g.n_bins, I.n_ang);
      b.mode = BP_PLAIN;
      b.alpha = alpha;
      b.beta = beta;
      if (ua) {
        const size_t npix = (size_t)I.g.n * I.g.n;
        b.mode = BP_UNROLL;
        b.u_in = I.image;
        b.img = ua->Uo + i * npix;
        b.x = ua->x;
        b.lam = ua->L + i * npix;
        b.scal = ua->scal;
      }
      b.chord = ctx->model;
      b.wg_begin = bw;
      bw += b.tiles_x * b.tiles_x;
      bj.push_back(b);
    }
    bp_wgs = bw;
  }
  plan.band = ctx->proj_band;
  plan.chord = ctx->model == 1;
  // one table: projection jobs, then reduction jobs; or backprojection jobs
  const size_t pbytes = pj.size() * sizeof(ProjJob), rbytes = rj.size() * sizeof(ProjJob);
  const size_t total = kind == 0 ? pbytes + rbytes : bj.size() * sizeof(BPJob);
  int slot = 0;
  void* host = ctx->ring.acquire(total, slot);
  if (!host || !ctx->btable.ensure(total)) return ctx->fail(TOMO_ENOMEM, "batch job table allocation failed");
  if (kind == 0) {
    std::memcpy(host, pj.data(), pbytes);
    if (rbytes) std::memcpy(static_cast<char*>(host) + pbytes, rj.data(), rbytes);
  } else {
    std::memcpy(host, bj.data(), total);
  }
  if (hipMemcpyAsync(ctx->btable.p, host, total, hipMemcpyHostToDevice, (hipStream_t)stream) != hipSuccess ||
      !ctx->ring.mark(slot, (hipStream_t)stream))
    return ctx->fail(TOMO_EDEVICE, "job table upload failed");
  plan.pjobs = static_cast<const ProjJob*>(ctx->btable.p);
  plan.rjobs = reinterpret_cast<const ProjJob*>(static_cast<const char*>(ctx->btable.p) + pbytes);
  return TOMO_OK;
}

// Argument checks of a batch: valid items, and no output overlapping any
// item's input or another item's output.
int check_items(tomo_ctx* ctx, const tomo_proj_item* items, int n_items, int kind) {
  if (!items || n_items < 1) return ctx->fail(TOMO_EINVAL, "empty item list");
  for (int i = 0; i < n_items; ++i) {
    const tomo_proj_item& I = items[i];
    if (int rc = check_geom(ctx, I.g)) return rc;
    if (I.n_ang < 1) return ctx->fail(TOMO_EINVAL, "item without angles");
    if (!I.angles || !I.image || !I.sino) return ctx->fail(TOMO_EINVAL, "null item pointer");
  }
  auto img_bytes = [](const tomo_proj_item& I) { return (size_t)I.g.n * I.g.n * 4; };
  auto sino_bytes = [](const tomo_proj_item& I) { return (size_t)I.n_ang * I.g.n_bins * 4; };
  for (int i = 0; i < n_items; ++i) {
    const void* out = kind == 0 ? (const void*)items[i].sino : (const void*)items[i].image;
    const size_t ob = kind == 0 ? sino_bytes(items[i]) : img_bytes(items[i]);
    for (int j = 0; j < n_items; ++j) {
      const void* in = kind == 0 ? (const void*)items[j].image : (const void*)items[j].sino;
      const size_t ib = kind == 0 ? img_bytes(items[j]) : sino_bytes(items[j]);
      if (overlaps(out, ob, in, ib)) return ctx->fail(TOMO_EINVAL, "an output overlaps an input");
      if (j != i) {
        const void* o2 = kind == 0 ? (const void*)items[j].sino : (const void*)items[j].image;
        const size_t b2 = kind == 0 ? sino_bytes(items[j]) : img_bytes(items[j]);
        if (overlaps(out, ob, o2, b2)) return ctx->fail(TOMO_EINVAL, "two outputs overlap");
      }
    }
  }
  return TOMO_OK;
}

bool same_msg(const std::vector<tomo_msg>& k, const tomo_msg* msg, int n) {
  if (!msg) return k.empty();
  return (int)k.size() == n && std::memcmp(k.data(), msg, sizeof(tomo_msg) * n) == 0;
}

bool same_regs(const std::vector<tomo_reg>& k, const tomo_reg* regs, int n) {
  return (int)k.size() == n && (n == 0 || std::memcmp(k.data(), regs, sizeof(tomo_reg) * n) == 0);
}

// the block of a slice, or null
const tomo_reg* reg_of(const tomo_reg* regs, int n_regs, int slice) {
  for (int r = 0; r < n_regs; ++r)
    if (regs[r].slice == slice) return &regs[r];
  return nullptr;
}

// Validates a block array against the node list; fills the image and side of
// each block's slice.
int check_regs(tomo_ctx* ctx, const tomo_node* nodes, int n_nodes, const tomo_reg* regs, int n_regs,
               std::vector<const float*>& xs, std::vector<int>& ns) {
  if (n_regs < 0 || (n_regs > 0 && !regs)) return ctx->fail(TOMO_EINVAL, "bad regularization block array");
  xs.assign(n_regs, nullptr);
  ns.assign(n_regs, 0);
  for (int r = 0; r < n_regs; ++r) {
    const tomo_reg& R = regs[r];
    for (int q = 0; q < r; ++q)
      if (regs[q].slice == R.slice) return ctx->fail(TOMO_EINVAL, "two regularization blocks for one slice");
    for (int i = 0; i < n_nodes; ++i)
      if (nodes[i].slice == R.slice) { xs[r] = nodes[i].x; ns[r] = nodes[i].g.n; break; }
    if (!xs[r]) return ctx->fail(TOMO_EINVAL, "regularization block of a slice no listed node has");
    if (R.kind != TOMO_REG_TIKHONOV && R.kind != TOMO_REG_TV) return ctx->fail(TOMO_EINVAL, "unknown regularizer");
    if (!(R.rho > 0.f) || !(R.mu >= 0.f)) return ctx->fail(TOMO_EINVAL, "regularization needs rho > 0 and mu >= 0");
    if (R.kind == TOMO_REG_TV && (!(R.tau > 0.f) || R.tau > 0.25f || R.tv_iters < 0 || R.tv_iters > 10000))
      return ctx->fail(TOMO_EINVAL, "TV needs 0 < tau <= 0.25 and 0 <= tv_iters <= 10000");
    if (!R.z || !R.nu || !R.tz || (R.kind == TOMO_REG_TV && !R.p))
      return ctx->fail(TOMO_EINVAL, "null regularization pointer");
    const size_t img = (size_t)ns[r] * ns[r] * sizeof(float);
    const void* ptr[5] = {R.z, R.nu, R.tz, xs[r], R.p};
    const size_t len[5] = {img, img, img, img, 2 * img};
    const int np = R.kind == TOMO_REG_TV ? 5 : 4;
    for (int a = 0; a < np; ++a)
      for (int b = a + 1; b < np; ++b)
        if (overlaps(ptr[a], len[a], ptr[b], len[b]))
          return ctx->fail(TOMO_EINVAL, "regularization arrays must not overlap each other or x");
  }
  return TOMO_OK;
}

RegPlan* get_reg_plan(tomo_ctx* ctx, const tomo_reg* regs, int n_regs, const std::vector<const float*>& xs,
                      const std::vector<int>& ns, int& rc) {
  rc = TOMO_OK;
  for (auto& p : ctx->rplans)
    if (same_regs(p->key, regs, n_regs) && p->xs == xs && p->ns == ns) return p.get();
  auto plan = std::make_unique<RegPlan>();
  plan->key.assign(regs, regs + n_regs);
  plan->xs = xs;
  plan->ns = ns;
  size_t scratch = 0;
  for (int r = 0; r < n_regs; ++r)
    if (regs[r].kind == TOMO_REG_TV) scratch += 2 * (size_t)ns[r] * ns[r];
  if (!plan->scratch.ensure(std::max<size_t>(scratch, 1) * sizeof(float)) ||
      !plan->jobs.ensure((size_t)std::max(n_regs, 1) * sizeof(RegJob))) {
    rc = ctx->fail(TOMO_ENOMEM, "regularization plan allocation failed");
    return nullptr;
  }
  std::vector<RegJob> jobs;
  float* sp = static_cast<float*>(plan->scratch.p);
  int w = 0;
  for (int r = 0; r < n_regs; ++r) {
    const tomo_reg& R = regs[r];
    RegJob j{};
    j.x = xs[r]; j.nu = R.nu; j.z = R.z; j.tz = R.tz;
    j.n = ns[r];
    j.kind = R.kind == TOMO_REG_TV ? REG_TV : REG_TIKHONOV;
    j.theta = R.mu / R.rho;
    j.irho_z = 1.f / R.rho;
    j.tau = R.tau;
    // with theta = 0 the prox is the identity: no iterations
    j.iters = (j.kind == REG_TV && j.theta > 0.f) ? R.tv_iters : 0;
    if (j.kind == REG_TV) {
      j.p[0] = R.p;
      j.p[1] = sp;
      sp += 2 * (size_t)ns[r] * ns[r];
      plan->launches = std::max(plan->launches, tv_launches(j.iters));
    }
    j.wg_begin = w;
    w += ((ns[r] + TV_TILE_H - 1) / TV_TILE_H) * ((ns[r] + TV_TILE_W - 1) / TV_TILE_W);   // one workgroup per tile
    jobs.push_back(j);
  }
  if (n_regs > 0 &&
      hipMemcpy(plan->jobs.p, jobs.data(), jobs.size() * sizeof(RegJob), hipMemcpyHostToDevice) != hipSuccess) {
    rc = ctx->fail(TOMO_EDEVICE, "regularization plan upload failed");
    return nullptr;
  }
  plan->n_jobs = n_regs;
  plan->wgs = w;
  ctx->rplans.push_back(std::move(plan));
  return ctx->rplans.back().get();
}

ConsPlan* get_cons_plan(tomo_ctx* ctx, const tomo_node* nodes, int n_nodes, const tomo_msg* msg,
                        const tomo_reg* regs, int n_regs, int& rc) {
  rc = TOMO_OK;
  uint64_t h = cons_hash(nodes, n_nodes, msg);
  if (n_regs > 0) h = hash_bytes(regs, sizeof(tomo_reg) * n_regs, h);
  auto range = ctx->cindex.equal_range(h);
  for (auto it = range.first; it != range.second; ++it)
    if (same_nodes(it->second->key, nodes, n_nodes) && same_msg(it->second->msg_key, msg, n_nodes) &&
        same_regs(it->second->reg_key, regs, n_regs))
      return it->second;
  auto plan = std::make_unique<ConsPlan>();
  plan->key.assign(nodes, nodes + n_nodes);
  if (msg) plan->msg_key.assign(msg, msg + n_nodes);
  if (n_regs > 0) plan->reg_key.assign(regs, regs + n_regs);
  std::vector<SegJob> seg;
  std::vector<AvgJob> avg;
  std::vector<NodeRef> refs;
  int aw = 0, dw = 0;
  for (int i = 0; i < n_nodes; ++i) {
    const tomo_node& N = nodes[i];
    const tomo_reg* B = reg_of(regs, n_regs, N.slice);
    SegJob s{};
    s.x = N.x; s.u = N.u; s.lam = N.lam;
    s.tz = B ? B->tz : nullptr;
    s.rho_z = B ? B->rho : 0.f;
    s.n = N.g.n; s.row0 = N.seg_row0; s.rows = N.seg_rows;
    s.rho = N.rho; s.eta2 = N.eta2;
    if (msg) {
      s.labels = msg[i].labels; s.centroids = msg[i].centroids; s.iters = msg[i].iters;
      s.coeffs = msg[i].coeffs; s.lohi = msg[i].lohi; s.xt = msg[i].x_tilde;
      plan->any_xt = plan->any_xt || s.xt;
    }
    s.src = N.x + (size_t)N.seg_row0 * N.g.n;
    s.dst = N.x + (size_t)N.seg_row0 * N.g.n;
    s.cols = s.ld = N.g.n;
    s.chunk_rows = dct_chunk_rows(N.seg_rows, N.g.n);
    s.n_chunks = (N.seg_rows + s.chunk_rows - 1) / s.chunk_rows;
    s.range_wg = plan->dct_range_wgs;
    s.code_wg = plan->dct_code_wgs;
    plan->dct_range_wgs += s.n_chunks;
    plan->dct_code_wgs += dct_code_wgs(N.seg_rows, N.g.n);
    seg.push_back(s);
    NodeRef r{};
    r.u = N.u; r.lam = N.lam; r.x = N.x; r.n = N.g.n; r.rho = N.rho;
    r.wg_begin = dw;
    dw += (int)(((long long)N.g.n * N.g.n + 1023) / 1024);      // k_dual: four values per thread
    refs.push_back(r);
    if (i == 0 || nodes[i - 1].slice != N.slice) {
      AvgJob a{};
      a.x = N.x; a.node0 = i; a.n_nodes = 0; a.n = N.g.n; a.wg_begin = aw;
      a.tz = B ? B->tz : nullptr;
      a.rho_z = B ? B->rho : 0.f;
      aw += (int)(((long long)N.g.n * N.g.n + 255) / 256);
      avg.push_back(a);
    }
    avg.back().n_nodes++;
  }
  // dual update of every block: nu += rho_z (z - x), as one more (u, lambda) entry
  for (int r = 0; r < n_regs; ++r) {
    const tomo_reg& R = regs[r];
    NodeRef ref{};
    for (int i = 0; i < n_nodes; ++i)
      if (nodes[i].slice == R.slice) { ref.x = nodes[i].x; ref.n = nodes[i].g.n; break; }
    ref.u = R.z; ref.lam = R.nu; ref.rho = R.rho;
    ref.wg_begin = dw;
    dw += (int)(((long long)ref.n * ref.n + 1023) / 1024);
    refs.push_back(ref);
  }
  // K-means jobs: segments that fit the registers first, then the longer ones,
  // each with its own slice of the workspace (labels are written only where the
  // caller asks for them)
  std::vector<KMJob> km_small, km_big;
  std::vector<KMBlock> kb_small, kb_big;
  std::vector<size_t> work_off(n_nodes, 0);
  size_t work_elems = 0;
  for (int i = 0; i < n_nodes; ++i) {
    const long long segn = (long long)nodes[i].seg_rows * nodes[i].g.n;
    if (segn > KM_LDS_VALUES) {
      work_off[i] = work_elems;
      work_elems += (size_t)(segn + 63) / 64 * 64;
    }
  }
  plan->dct_range_uni = seg.empty() ? 0 : seg[0].n_chunks;
  plan->dct_code_uni = seg.empty() ? 0 : dct_code_wgs(seg[0].rows, seg[0].n);
  for (const auto& j : seg) {
    if (j.n_chunks != plan->dct_range_uni) plan->dct_range_uni = 0;
    if (dct_code_wgs(j.rows, j.n) != plan->dct_code_uni) plan->dct_code_uni = 0;
  }
  if (!plan->dctpart.ensure((size_t)plan->dct_range_wgs * sizeof(float4))) {
    rc = ctx->fail(TOMO_ENOMEM, "consensus plan allocation failed");
    return nullptr;
  }
  {
    float4* part = static_cast<float4*>(plan->dctpart.p);
    for (auto& s : seg) s.part = part + s.range_wg;
  }
  if (!plan->seg.ensure(seg.size() * sizeof(SegJob)) || !plan->avg.ensure(avg.size() * sizeof(AvgJob)) ||
      !plan->noderefs.ensure(refs.size() * sizeof(NodeRef)) ||
      !plan->kmjobs.ensure((size_t)n_nodes * sizeof(KMJob)) ||
      !plan->kmwork.ensure(work_elems * sizeof(float))) {
    rc = ctx->fail(TOMO_ENOMEM, "consensus plan allocation failed");
    return nullptr;
  }
  for (int i = 0; i < n_nodes; ++i) {
    const tomo_node& N = nodes[i];
    size_t off = (size_t)N.seg_row0 * N.g.n;
    KMJob j{};
    j.src = N.x + off;
    j.x = N.x + off;
    j.a_hat = N.x + off;
    j.u = N.u + off;
    j.lam = N.lam + off;
    KMBlock kb{nullptr, 0.f};
    if (const tomo_reg* B = reg_of(regs, n_regs, N.slice)) {
      kb.tz = B->tz + off;
      kb.rho_z = B->rho;
    }
    j.n = (long long)N.seg_rows * N.g.n;
    j.rho = N.rho;
    j.eta2 = N.eta2;
    j.labels = msg ? msg[i].labels : nullptr;
    j.cent = msg ? msg[i].centroids : nullptr;
    j.iters = msg ? msg[i].iters : nullptr;
    j.xt = msg ? msg[i].x_tilde : nullptr;
    if (j.n > KM_LDS_VALUES) {
      j.work = static_cast<float*>(plan->kmwork.p) + work_off[i];
      km_big.push_back(j);
      kb_big.push_back(kb);
    } else {
      km_small.push_back(j);
      kb_small.push_back(kb);
    }
  }
  plan->km_small = (int)km_small.size();
  plan->km_big = (int)km_big.size();
  km_small.insert(km_small.end(), km_big.begin(), km_big.end());
  kb_small.insert(kb_small.end(), kb_big.begin(), kb_big.end());
  if (n_regs > 0 &&
      (!plan->kmblocks.ensure(kb_small.size() * sizeof(KMBlock)) ||
       hipMemcpy(plan->kmblocks.p, kb_small.data(), kb_small.size() * sizeof(KMBlock), hipMemcpyHostToDevice) !=
           hipSuccess)) {
    rc = ctx->fail(TOMO_EDEVICE, "K-means block table upload failed");
    return nullptr;
  }
  if (hipMemcpy(plan->kmjobs.p, km_small.data(), km_small.size() * sizeof(KMJob), hipMemcpyHostToDevice) !=
      hipSuccess) {
    rc = ctx->fail(TOMO_EDEVICE, "K-means plan upload failed");
    return nullptr;
  }
  if (hipMemcpy(plan->seg.p, seg.data(), seg.size() * sizeof(SegJob), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(plan->avg.p, avg.data(), avg.size() * sizeof(AvgJob), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(plan->noderefs.p, refs.data(), refs.size() * sizeof(NodeRef), hipMemcpyHostToDevice) != hipSuccess) {
    rc = ctx->fail(TOMO_EDEVICE, "descriptor upload failed");
    return nullptr;
  }
  plan->n_seg = (int)seg.size();
  plan->n_refs = (int)refs.size();
  plan->n_avg = (int)avg.size();
  plan->avg_wgs = aw;
  plan->dual_wgs = dw;
  ctx->cindex.emplace(h, plan.get());
  ctx->cplans.push_back(std::move(plan));
  return ctx->cplans.back().get();
}

}  // namespace

extern "C" {

const char* tomo_status_string(int status) {
  switch (status) {
    case TOMO_OK: return "ok";
    case TOMO_EINVAL: return "invalid argument";
    case TOMO_ENOMEM: return "out of device memory";
    case TOMO_EDEVICE: return "device error";
    case TOMO_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* tomo_last_error(const tomo_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int tomo_create(tomo_ctx** out, int device) {
  if (!out) return TOMO_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TOMO_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TOMO_EDEVICE;
  tomo_ctx* c = new (std::nothrow) tomo_ctx();
  if (!c) return TOMO_ENOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = std::max(1, prop.multiProcessorCount);
  int xcc = 1;
  if (hipDeviceGetAttribute(&xcc, hipDeviceAttributeNumberOfXccs, device) == hipSuccess) c->n_xcc = std::max(1, xcc);
  (void)hipGetLastError();
  if (int rc = resolve_scratch(device)) {
    delete c;
    return rc;
  }
  *out = c;
  return TOMO_OK;
}

int tomo_destroy(tomo_ctx* ctx) {
  if (!ctx) return TOMO_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
  return TOMO_OK;
}

int tomo_set_option(tomo_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return TOMO_EINVAL;
  switch (option) {
    case TOMO_OPT_PROJ_JOB_WGS:
      if (value < 1 || value > 65536) return ctx->fail(TOMO_EINVAL, "projector workgroups per job out of range");
      ctx->proj_job_wgs = (int)value;
      break;
    case TOMO_OPT_PROJ_BAND:
      if (value != 16 && value != 32) return ctx->fail(TOMO_EINVAL, "projector band depth must be 16 or 32");
      ctx->proj_band = (int)value;
      break;
    case TOMO_OPT_PROJ_KERNEL:
      if (value != 0 && value != 1) return ctx->fail(TOMO_EINVAL, "projector kernel must be 0 or 1");
      ctx->proj_kernel = (int)value;
      break;
    case TOMO_OPT_PROJ_MODEL:
      if (value != 0 && value != 1) return ctx->fail(TOMO_EINVAL, "projector model must be 0 or 1");
      ctx->model = (int)value;
      break;
    case TOMO_OPT_PROJ_ORDER:
      if (value < 0 || value > 2) return ctx->fail(TOMO_EINVAL, "projector order must be 0, 1 or 2");
      ctx->proj_order = (int)value;
      break;
    default:
      return ctx->fail(TOMO_EINVAL, "unknown option");
  }
  for (auto& p : ctx->lplans) ctx->retired_l.push_back(std::move(p));
  for (auto& p : ctx->cplans) ctx->retired_c.push_back(std::move(p));
  ctx->lplans.clear();
  ctx->cplans.clear();
  ctx->lindex.clear();
  ctx->cindex.clear();
  return TOMO_OK;
}

int tomo_release(tomo_ctx* ctx) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = set_device(ctx)) return rc;
  if (hipDeviceSynchronize() != hipSuccess) return ctx->fail(TOMO_EDEVICE, "hipDeviceSynchronize failed");
  ctx->lplans.clear();
  ctx->cplans.clear();
  ctx->retired_l.clear();
  ctx->retired_c.clear();
  ctx->rplans.clear();
  ctx->lindex.clear();
  ctx->cindex.clear();
  for (DevBuf* b : {&ctx->partial, &ctx->pbbase, &ctx->km_work, &ctx->dct_part, &ctx->unroll_part, &ctx->ctr_resid,
                    &ctx->ecode_off, &ctx->btable, &ctx->bpartial, &ctx->bbbase})
    b->release();
  return TOMO_OK;
}

int tomo_project(tomo_ctx* ctx, tomo_geom g, const double* angles, int32_t n_ang, const float* image,
                 float* sino, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = check_geom(ctx, g)) return rc;
  if (n_ang < 0) return ctx->fail(TOMO_EINVAL, "n_ang < 0");
  if (n_ang == 0) return TOMO_OK;
  if (!angles || !image || !sino) return ctx->fail(TOMO_EINVAL, "null pointer");
  if (overlaps(image, (size_t)g.n * g.n * 4, sino, (size_t)n_ang * g.n_bins * 4))
    return ctx->fail(TOMO_EINVAL, "image and sino overlap");
  if (int rc = set_device(ctx)) return rc;
  if (int rc = project_one(ctx, g, angles, n_ang, image, nullptr, sino, stream)) return rc;
  return launch_status(ctx, "tomo_project");
}

int tomo_backproject(tomo_ctx* ctx, tomo_geom g, const double* angles, int32_t n_ang, const float* sino,
                     float* image, float alpha, float beta, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = check_geom(ctx, g)) return rc;
  if (n_ang < 0) return ctx->fail(TOMO_EINVAL, "n_ang < 0");
  if (!image || (n_ang > 0 && (!angles || !sino))) return ctx->fail(TOMO_EINVAL, "null pointer");
  if (n_ang > 0 && overlaps(image, (size_t)g.n * g.n * 4, sino, (size_t)n_ang * g.n_bins * 4))
    return ctx->fail(TOMO_EINVAL, "image and sino overlap");
  if (int rc = set_device(ctx)) return rc;
  BPJob j = make_bp_job(sino, angles, image, g.n, g.n_bins, n_ang);
  j.mode = BP_PLAIN;
  j.alpha = alpha;
  j.beta = beta;
  j.chord = ctx->model;
  launch_backproject(Single<BPJob>{j}, j.tiles_x * j.tiles_x, j.chord, stream);
  return launch_status(ctx, "tomo_backproject");
}

int tomo_project_many(tomo_ctx* ctx, const tomo_proj_item* items, int32_t n_items, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = check_items(ctx, items, n_items, 0)) return rc;
  if (int rc = set_device(ctx)) return rc;
  ProjLaunch L;
  int unused = 0;
  if (int rc = stage_batch(ctx, items, n_items, 0, 0.f, 0.f, stream, L, unused)) return rc;
  launch_projection(L, stream);
  return launch_status(ctx, "tomo_project_many");
}

int tomo_backproject_many(tomo_ctx* ctx, const tomo_proj_item* items, int32_t n_items, float alpha, float beta,
                          void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = check_items(ctx, items, n_items, 1)) return rc;
  if (int rc = set_device(ctx)) return rc;
  ProjLaunch L;
  int wgs = 0;
  if (int rc = stage_batch(ctx, items, n_items, 1, alpha, beta, stream, L, wgs)) return rc;
  launch_backproject(Many<BPJob>{static_cast<const BPJob*>(ctx->btable.p), n_items}, wgs, ctx->model, stream);
  return launch_status(ctx, "tomo_backproject_many");
}

int tomo_unroll_local_step(tomo_ctx* ctx, const tomo_proj_item* items, int32_t n_items, const float* D,
                           const float* x, const float* L, const float* scal, float* Uo, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = check_items(ctx, items, n_items, 0)) return rc;
  if (!D || !x || !L || !scal || !Uo) return ctx->fail(TOMO_EINVAL, "null pointer");
  const int n = items[0].g.n, nb = items[0].g.n_bins;
  size_t rows = 0;
  for (int i = 0; i < n_items; ++i) {
    if (items[i].g.n != n || items[i].g.n_bins != nb) return ctx->fail(TOMO_EINVAL, "items must share n and n_bins");
    rows += items[i].n_ang;
  }
  const size_t img = (size_t)n * n * 4, stack = img * n_items, dbytes = rows * nb * 4;
  // R_i rows (first launch) and Uo (second) against every operand
  for (int i = 0; i < n_items; ++i) {
    const size_t sb = (size_t)items[i].n_ang * nb * 4;
    if (overlaps(items[i].sino, sb, D, dbytes) || overlaps(items[i].sino, sb, x, img) ||
        overlaps(items[i].sino, sb, L, stack) || overlaps(items[i].sino, sb, scal, 8) ||
        overlaps(Uo, stack, items[i].image, img) || overlaps(Uo, stack, items[i].sino, sb))
      return ctx->fail(TOMO_EINVAL, "an output overlaps an input or the other output");
  }
  if (overlaps(Uo, stack, D, dbytes) || overlaps(Uo, stack, x, img) || overlaps(Uo, stack, L, stack) ||
      overlaps(Uo, stack, scal, 8))
    return ctx->fail(TOMO_EINVAL, "Uo overlaps an input");
  if (int rc = set_device(ctx)) return rc;
  const UnrollArgs ua{D, x, L, scal, Uo};
  ProjLaunch P;
  int unused = 0;
  if (int rc = stage_batch(ctx, items, n_items, 0, 0.f, 0.f, stream, P, unused, &ua)) return rc;
  launch_projection(P, stream);
  ProjLaunch B;
  int wgs = 0;
  if (int rc = stage_batch(ctx, items, n_items, 1, 1.f, 0.f, stream, B, wgs, &ua)) return rc;
  launch_backproject(Many<BPJob>{static_cast<const BPJob*>(ctx->btable.p), n_items}, wgs, ctx->model, stream);
  return launch_status(ctx, "tomo_unroll_local_step");
}

int tomo_ctr_gd(tomo_ctx* ctx, tomo_geom g, const double* angles, int32_t n_ang, const float* d, float* u,
                float eta, int32_t iters, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (int rc = check_geom(ctx, g)) return rc;
  if (n_ang < 1) return ctx->fail(TOMO_EINVAL, "n_ang < 1");
  if (iters < 0) return ctx->fail(TOMO_EINVAL, "iters < 0");
  if (!std::isfinite(eta)) return ctx->fail(TOMO_EINVAL, "eta must be finite");
  if (!angles || !d || !u) return ctx->fail(TOMO_EINVAL, "null pointer");
  const size_t img = (size_t)g.n * g.n * 4, sino = (size_t)n_ang * g.n_bins * 4;
  if (overlaps(u, img, d, sino)) return ctx->fail(TOMO_EINVAL, "u and d overlap");
  if (iters == 0) return TOMO_OK;
  if (int rc = set_device(ctx)) return rc;
  if (!ctx->ctr_resid.ensure(sino)) return ctx->fail(TOMO_ENOMEM, "workspace");
  float* r = static_cast<float*>(ctx->ctr_resid.p);
  BPJob b = make_bp_job(r, angles, u, g.n, g.n_bins, n_ang);
  b.mode = BP_PLAIN;
  b.alpha = -eta;
  b.beta = 1.f;
  b.chord = ctx->model;
  for (int it = 0; it < iters; ++it) {
    if (int rc = project_one(ctx, g, angles, n_ang, u, d, r, stream)) return rc;     // r = P u - d
    launch_backproject(Single<BPJob>{b}, b.tiles_x * b.tiles_x, b.chord, stream);   // u -= eta P^T r
  }
  return launch_status(ctx, "tomo_ctr_gd");
}

int admm_local_update(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t e1, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (e1 < 0) return ctx->fail(TOMO_EINVAL, "E1 < 0");
  if (!nodes || n_nodes < 1) return ctx->fail(TOMO_EINVAL, "empty node list");
  if (int rc = set_device(ctx)) return rc;
  int rc = TOMO_OK;
  LocalPlan* plan = find_local_plan(ctx, nodes, n_nodes);
  if (!plan) {
    if (int rc2 = check_nodes(ctx, nodes, n_nodes)) return rc2;
    plan = get_local_plan(ctx, nodes, n_nodes, rc);
  }
  if (!plan) return rc;
  Many<BPJob> bs{static_cast<const BPJob*>(plan->bjobs.p), plan->n_b};
  if (plan->b_ordered) bs.order = static_cast<const int2*>(plan->border.p);
  for (int e = 0; e < e1; ++e) {
    launch_projection(launch_of(plan), stream);
    launch_backproject(bs, plan->b_wgs, plan->chord, stream);
  }
  return launch_status(ctx, "admm_local_update");
}

int admm_local_phase(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t phase, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (phase != 0 && phase != 1) return ctx->fail(TOMO_EINVAL, "phase must be 0 or 1");
  if (!nodes || n_nodes < 1) return ctx->fail(TOMO_EINVAL, "empty node list");
  if (int rc = set_device(ctx)) return rc;
  int rc = TOMO_OK;
  LocalPlan* plan = find_local_plan(ctx, nodes, n_nodes);
  if (!plan) {
    if (int rc2 = check_nodes(ctx, nodes, n_nodes)) return rc2;
    plan = get_local_plan(ctx, nodes, n_nodes, rc);
  }
  if (!plan) return rc;
  if (phase == 0) {
    launch_projection(launch_of(plan), stream);
  } else {
    Many<BPJob> bs{static_cast<const BPJob*>(plan->bjobs.p), plan->n_b};
    if (plan->b_ordered) bs.order = static_cast<const int2*>(plan->border.p);
    launch_backproject(bs, plan->b_wgs, plan->chord, stream);
  }
  return launch_status(ctx, "admm_local_phase");
}

int admm_consensus(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t mode, int32_t e2,
                   const tomo_quant* q, const tomo_msg* msg, void* stream) {
  return admm_consensus_reg(ctx, nodes, n_nodes, mode, e2, q, msg, nullptr, 0, stream);
}

int admm_consensus_reg(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, int32_t mode, int32_t e2,
                       const tomo_quant* q, const tomo_msg* msg, const tomo_reg* regs, int32_t n_regs,
                       void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (mode != TOMO_XUPDATE_SEGMENT && mode != TOMO_XUPDATE_AVERAGE) return ctx->fail(TOMO_EINVAL, "bad mode");
  if (e2 < 0) return ctx->fail(TOMO_EINVAL, "E2 < 0");
  if (int rc = check_nodes(ctx, nodes, n_nodes)) return rc;
  int kind = q ? q->kind : TOMO_QUANT_NONE;
  if (kind < TOMO_QUANT_NONE || kind > TOMO_QUANT_DCT) return ctx->fail(TOMO_EINVAL, "bad quantizer");
  for (int i = 0; i < n_nodes; ++i) {
    long long segn = (long long)nodes[i].seg_rows * nodes[i].g.n;
    if (kind == TOMO_QUANT_KMEANS && (q->levels < 1 || q->levels > 256 || q->max_iter < 0 || segn >= (1ll << 31)))
      return ctx->fail(TOMO_EINVAL, "bad K-means parameters");
    if (kind == TOMO_QUANT_DCT && (q->quality < 1 || q->quality > 100 || nodes[i].seg_rows % 8 || nodes[i].g.n % 8))
      return ctx->fail(TOMO_EINVAL, "bad DCT parameters (quality 1..100, segment sides multiples of 8)");
  }
  std::vector<const float*> rxs;
  std::vector<int> rns;
  if (int rc = check_regs(ctx, nodes, n_nodes, regs, n_regs, rxs, rns)) return rc;
  if (int rc = set_device(ctx)) return rc;
  int rc = TOMO_OK;
  ConsPlan* plan = get_cons_plan(ctx, nodes, n_nodes, msg, regs, n_regs, rc);
  if (!plan) return rc;
  hipStream_t s = (hipStream_t)stream;
  const SegJob* seg = static_cast<const SegJob*>(plan->seg.p);
  const NodeRef* refs = static_cast<const NodeRef*>(plan->noderefs.p);
  const int do_x = mode == TOMO_XUPDATE_SEGMENT;
  if (mode == TOMO_XUPDATE_AVERAGE) {
    Many<AvgJob> as{static_cast<const AvgJob*>(plan->avg.p), plan->n_avg};
    hipLaunchKernelGGL(k_avg, dim3(plan->avg_wgs), dim3(256), 0, s, as, refs);
  }
  if (kind == TOMO_QUANT_KMEANS) {
    // the x-update (SEG) runs inside the K-means kernel; AVG already wrote x
    const KMJob* kj = static_cast<const KMJob*>(plan->kmjobs.p);
    const KMBlock* kb = plan->reg_key.empty() ? nullptr : static_cast<const KMBlock*>(plan->kmblocks.p);
    const int ex = do_x ? e2 : 0;
    if (plan->km_small > 0)
      hipLaunchKernelGGL((plan->reg_key.empty() ? k_kmeans<true, false> : k_kmeans<true, true>), dim3(plan->km_small),
                         dim3(kKmThreads), 0, s, kj, KMJob{}, q->levels, q->max_iter, ex, kb);
    if (plan->km_big > 0)
      hipLaunchKernelGGL((plan->reg_key.empty() ? k_kmeans<false, false> : k_kmeans<false, true>), dim3(plan->km_big),
                         dim3(kKmThreads), 0, s, kj + plan->km_small, KMJob{}, q->levels, q->max_iter, ex,
                         kb ? kb + plan->km_small : nullptr);
  } else if (kind == TOMO_QUANT_DCT) {
    hipLaunchKernelGGL(k_dct_range, dim3(plan->dct_range_wgs), dim3(DCT_THREADS), 0, s, seg, plan->n_seg,
                       plan->dct_range_uni, SegJob{}, do_x, e2);
    hipLaunchKernelGGL(k_dct_code, dim3(plan->dct_code_wgs), dim3(DCT_THREADS), 0, s, seg, plan->n_seg,
                       plan->dct_code_uni, SegJob{}, q->quality);
  } else if (do_x || plan->any_xt) {
    hipLaunchKernelGGL(k_seg_none, dim3(plan->n_seg), dim3(256), 0, s, seg, do_x, e2);
  }
  Many<NodeRef> ds{refs, plan->n_refs};
  hipLaunchKernelGGL(k_dual, dim3(plan->dual_wgs), dim3(256), 0, s, ds);
  return launch_status(ctx, "admm_consensus");
}

int admm_reg_update(tomo_ctx* ctx, const tomo_node* nodes, int32_t n_nodes, const tomo_reg* regs, int32_t n_regs,
                    void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (!nodes || n_nodes < 1) return ctx->fail(TOMO_EINVAL, "empty node list");
  if (n_regs == 0) return TOMO_OK;
  std::vector<const float*> xs;
  std::vector<int> ns;
  if (int rc = check_regs(ctx, nodes, n_nodes, regs, n_regs, xs, ns)) return rc;
  if (int rc = set_device(ctx)) return rc;
  int rc = TOMO_OK;
  RegPlan* plan = get_reg_plan(ctx, regs, n_regs, xs, ns, rc);
  if (!plan) return rc;
  hipStream_t s = (hipStream_t)stream;
  Many<RegJob> js{static_cast<const RegJob*>(plan->jobs.p), plan->n_jobs};
  for (int l = 0; l < plan->launches; ++l) hipLaunchKernelGGL(k_reg_step, dim3(plan->wgs), dim3(TV_THREADS), 0, s, js, l);
  return launch_status(ctx, "admm_reg_update");
}

int quantize_kmeans(tomo_ctx* ctx, const float* a, int64_t n, int32_t k, int32_t max_iter, uint8_t* labels,
                    float* centroids, float* a_hat, int32_t* iters, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (n < 1 || n >= (1ll << 31)) return ctx->fail(TOMO_EINVAL, "n must lie in [1, 2^31)");
  if (k < 1 || k > 256 || max_iter < 0) return ctx->fail(TOMO_EINVAL, "k must lie in [1, 256], max_iter >= 0");
  if (!a || !labels || !centroids) return ctx->fail(TOMO_EINVAL, "null pointer");
  if (a_hat && a_hat != a && overlaps(a, (size_t)n * 4, a_hat, (size_t)n * 4))
    return ctx->fail(TOMO_EINVAL, "a_hat partially overlaps a");
  if (int rc = set_device(ctx)) return rc;
  const bool big = n > KM_LDS_VALUES;
  if (big && !ctx->km_work.ensure((size_t)n * sizeof(float))) return ctx->fail(TOMO_ENOMEM, "workspace");
  KMJob j{};
  j.src = a;
  j.a_hat = a_hat;
  j.labels = labels;
  j.cent = centroids;
  j.iters = iters;
  j.n = n;
  j.rho = 1.f;
  if (big) {
    j.work = static_cast<float*>(ctx->km_work.p);
    hipLaunchKernelGGL((k_kmeans<false, false>), dim3(1), dim3(kKmThreads), 0, (hipStream_t)stream, nullptr, j, k, max_iter,
                       0, (const KMBlock*)nullptr);
  } else {
    hipLaunchKernelGGL((k_kmeans<true, false>), dim3(1), dim3(kKmThreads), 0, (hipStream_t)stream, nullptr, j, k, max_iter,
                       0, (const KMBlock*)nullptr);
  }
  return launch_status(ctx, "quantize_kmeans");
}

// Argument checks and the two launches of the DCT codec; `part` holds the range
// partials (null: the context's workspace, allocated on first use).
static int dct_codec(tomo_ctx* ctx, const float* a, int32_t rows, int32_t cols, int32_t ld, int32_t quality,
                     int16_t* coeffs, float* a_hat, float* lohi, float4* part, void* stream, const char* what) {
  if (!ctx) return TOMO_EINVAL;
  if (rows < 8 || cols < 8 || rows % 8 || cols % 8 || ld < cols)
    return ctx->fail(TOMO_EINVAL, "rows, cols must be positive multiples of 8 and ld >= cols");
  if (quality < 1 || quality > 100) return ctx->fail(TOMO_EINVAL, "quality must lie in [1, 100]");
  if (!a || !a_hat) return ctx->fail(TOMO_EINVAL, "null pointer");
  if (a_hat != a && overlaps(a, (size_t)rows * ld * 4, a_hat, (size_t)rows * ld * 4))
    return ctx->fail(TOMO_EINVAL, "a_hat partially overlaps a");
  if (int rc = set_device(ctx)) return rc;
  SegJob j{};
  j.src = a;
  j.dst = a_hat;
  j.rows = rows;
  j.cols = cols;
  j.ld = ld;
  j.coeffs = coeffs;
  j.lohi = lohi;
  j.rho = 1.f;
  j.chunk_rows = dct_chunk_rows(rows, cols);
  j.n_chunks = (rows + j.chunk_rows - 1) / j.chunk_rows;
  if (j.n_chunks > DCT_MAX_CHUNKS) return ctx->fail(TOMO_EINVAL, "more range partials than the scratch holds");
  if (!part) {
    if (!ctx->dct_part.ensure((size_t)DCT_MAX_CHUNKS * sizeof(float4))) return ctx->fail(TOMO_ENOMEM, "workspace");
    part = static_cast<float4*>(ctx->dct_part.p);
  }
  j.part = part;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_dct_range, dim3(j.n_chunks), dim3(DCT_THREADS), 0, s, nullptr, 1, 0, j, 0, 0);
  hipLaunchKernelGGL(k_dct_code, dim3(dct_code_wgs(rows, cols)), dim3(DCT_THREADS), 0, s, nullptr, 1, 0, j, quality);
  return launch_status(ctx, what);
}

int quantize_dct(tomo_ctx* ctx, const float* a, int32_t rows, int32_t cols, int32_t ld, int32_t quality,
                 int16_t* coeffs, float* a_hat, float* lohi, void* stream) {
  return dct_codec(ctx, a, rows, cols, ld, quality, coeffs, a_hat, lohi, nullptr, stream, "quantize_dct");
}

int quantize_dct_noalloc(tomo_ctx* ctx, const float* a, int32_t rows, int32_t cols, int32_t ld, int32_t quality,
                         int16_t* coeffs, float* a_hat, float* lohi, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  float4* part = scratch_of(ctx->device);
  if (!part) return ctx->fail(TOMO_EDEVICE, "device scratch not resolved");
  return dct_codec(ctx, a, rows, cols, ld, quality, coeffs, a_hat, lohi, part, stream, "quantize_dct_noalloc");
}

int tomo_pack_labels(tomo_ctx* ctx, const uint8_t* labels, int64_t n, int32_t bits, uint32_t* packed,
                     void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (bits < 1 || bits > 8) return ctx->fail(TOMO_EINVAL, "bits must be in [1, 8]");
  if (n < 0 || n >= (int64_t(1) << 31)) return ctx->fail(TOMO_EINVAL, "n must be in [0, 2^31)");
  if (n == 0) return TOMO_OK;
  if (!labels || !packed) return ctx->fail(TOMO_EINVAL, "null pointer");
  const long long words = (n * bits + 31) / 32;
  if (overlaps(labels, (size_t)n, packed, (size_t)words * 4)) return ctx->fail(TOMO_EINVAL, "labels and packed overlap");
  if (int rc = set_device(ctx)) return rc;
  hipLaunchKernelGGL(k_pack_labels, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, (hipStream_t)stream, labels,
                     (int)n, bits, packed, words);
  return launch_status(ctx, "tomo_pack_labels");
}

int tomo_unpack_labels(tomo_ctx* ctx, const uint32_t* packed, int64_t n, int32_t bits, const float* centroids,
                       int32_t k, uint8_t* labels, float* a_hat, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (bits < 1 || bits > 8) return ctx->fail(TOMO_EINVAL, "bits must be in [1, 8]");
  if (n < 0 || n >= (int64_t(1) << 31)) return ctx->fail(TOMO_EINVAL, "n must be in [0, 2^31)");
  if (a_hat && (!centroids || k < 1 || k > 256)) return ctx->fail(TOMO_EINVAL, "a_hat needs centroids and 1 <= k <= 256");
  if (n == 0 || (!labels && !a_hat)) return TOMO_OK;
  if (!packed) return ctx->fail(TOMO_EINVAL, "null pointer");
  const size_t words = (size_t)((n * bits + 31) / 32) * 4;
  if ((labels && overlaps(packed, words, labels, (size_t)n)) || (a_hat && overlaps(packed, words, a_hat, (size_t)n * 4)))
    return ctx->fail(TOMO_EINVAL, "outputs overlap the packed stream");
  if (int rc = set_device(ctx)) return rc;
  hipLaunchKernelGGL(k_unpack_labels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, packed,
                     (int)n, bits, centroids, a_hat ? k : 1, labels, a_hat);
  return launch_status(ctx, "tomo_unpack_labels");
}

int64_t tomo_dct_encode_words(int32_t rows, int32_t cols) {
  if (rows <= 0 || cols <= 0 || rows % 8 || cols % 8) return 0;
  const int64_t blocks = (int64_t)(rows / 8) * (cols / 8);
  return (blocks * ECODE_MAX_BITS + 31) / 32;
}

int tomo_dct_encode(tomo_ctx* ctx, const int16_t* coeffs, int32_t rows, int32_t cols, int32_t ld, uint32_t* words,
                    int64_t max_words, uint32_t* restart, uint32_t* total_bits, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (rows <= 0 || cols <= 0 || rows % 8 || cols % 8 || ld < cols)
    return ctx->fail(TOMO_EINVAL, "rows and cols must be positive multiples of 8 and ld >= cols");
  if (!coeffs || !words || !restart || !total_bits) return ctx->fail(TOMO_EINVAL, "null pointer");
  const int64_t blocks = (int64_t)(rows / 8) * (cols / 8);
  if (blocks * ECODE_MAX_BITS >= (int64_t(1) << 32))
    return ctx->fail(TOMO_EUNSUPPORTED, "segment too large for 32-bit bit offsets");
  const int64_t need = tomo_dct_encode_words(rows, cols);
  if (max_words < need) return ctx->fail(TOMO_EINVAL, "words holds fewer than tomo_dct_encode_words(rows, cols)");
  if (overlaps(coeffs, (size_t)rows * ld * 2, words, (size_t)need * 4))
    return ctx->fail(TOMO_EINVAL, "coeffs and words overlap");
  if (int rc = set_device(ctx)) return rc;
  if (!ctx->ecode_off.ensure((size_t)blocks * 4)) return ctx->fail(TOMO_ENOMEM, "workspace");
  unsigned* off = static_cast<unsigned*>(ctx->ecode_off.p);
  const int nb = (int)blocks, n_bc = cols / 8, grid = (nb + 255) / 256;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_ecode_zero, dim3((unsigned)std::min<int64_t>((need + 255) / 256, 4096)), dim3(256), 0, s, words,
                     (long long)need);
  hipLaunchKernelGGL(k_ecode_bits, dim3(grid), dim3(256), 0, s, coeffs, ld, n_bc, nb, off);
  hipLaunchKernelGGL(k_ecode_scan, dim3(1), dim3(1024), 0, s, off, nb, restart, total_bits);
  hipLaunchKernelGGL(k_ecode_write, dim3(grid), dim3(256), 0, s, coeffs, ld, n_bc, nb, off, words);
  return launch_status(ctx, "tomo_dct_encode");
}

int tomo_dct_decode(tomo_ctx* ctx, const uint32_t* words, int64_t n_words, const uint32_t* restart,
                    const uint32_t* total_bits, int32_t rows, int32_t cols, int32_t ld, int16_t* coeffs,
                    int32_t* status, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (rows <= 0 || cols <= 0 || rows % 8 || cols % 8 || ld < cols)
    return ctx->fail(TOMO_EINVAL, "rows and cols must be positive multiples of 8 and ld >= cols");
  if (!words || !restart || !total_bits || !coeffs) return ctx->fail(TOMO_EINVAL, "null pointer");
  if (n_words < 0) return ctx->fail(TOMO_EINVAL, "n_words < 0");
  if (overlaps(coeffs, (size_t)rows * ld * 2, words, (size_t)n_words * 4))
    return ctx->fail(TOMO_EINVAL, "coeffs and words overlap");
  if (int rc = set_device(ctx)) return rc;
  const int64_t blocks = (int64_t)(rows / 8) * (cols / 8);
  const int64_t intervals = (blocks + ECODE_INTERVAL - 1) / ECODE_INTERVAL;
  hipLaunchKernelGGL(k_ecode_decode, dim3((unsigned)((intervals + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     words, (long long)n_words, restart, total_bits, cols / 8, (int)blocks, coeffs, ld, status);
  return launch_status(ctx, "tomo_dct_decode");
}

int tomo_sqdiff(tomo_ctx* ctx, const float* a, const float* b, int64_t n, double* out, void* stream) {
  if (!ctx) return TOMO_EINVAL;
  if (n < 0 || !a || !b || !out) return ctx->fail(TOMO_EINVAL, "bad arguments");
  if (int rc = set_device(ctx)) return rc;
  hipLaunchKernelGGL(k_sqdiff, dim3(1), dim3(1024), 0, (hipStream_t)stream, a, b, (long long)n, out);
  return launch_status(ctx, "tomo_sqdiff");
}


// ---------------------------------------------------------------------------
// Unrolled (differentiable) ADMM: elementwise steps and their gradients
// ---------------------------------------------------------------------------
static constexpr int kUnrollThreads = 256;
static constexpr int kUnrollMaxWgs = 2048;     // workgroups of a reducing launch (one partial each)

static int unroll_wgs(long long items) {
  return (int)std::max(1LL, std::min<long long>(kUnrollMaxWgs, (items + kUnrollThreads - 1) / kUnrollThreads));
}

static int unroll_check(tomo_ctx* ctx, int32_t m, int64_t npix, std::initializer_list<const void*> ptrs) {
  if (!ctx) return TOMO_EINVAL;
  if (m < 1 || npix < 1 || (long long)m * npix >= (1ll << 40)) return ctx->fail(TOMO_EINVAL, "bad sizes");
  for (const void* p : ptrs)
    if (!p) return ctx->fail(TOMO_EINVAL, "null pointer");
  return set_device(ctx);
}

// two blocks of partials (u-step: A and B), each kUnrollMaxWgs * 3 doubles
static double* unroll_parts(tomo_ctx* ctx) {
  if (!ctx->unroll_part.ensure((size_t)2 * kUnrollMaxWgs * 3 * sizeof(double))) return nullptr;
  return static_cast<double*>(ctx->unroll_part.p);
}

int tomo_axpby(tomo_ctx* ctx, int64_t n, float alpha, const float* a, float beta, const float* b, float* out,
               void* stream) {
  if (int rc = unroll_check(ctx, 1, n, {a, b, out})) return rc;
  hipLaunchKernelGGL(k_axpby, dim3(unroll_wgs(n)), dim3(kUnrollThreads), 0, (hipStream_t)stream, (long long)n, alpha,
                     a, beta, b, out);
  return launch_status(ctx, "tomo_axpby");
}

int tomo_unroll_ustep(tomo_ctx* ctx, int32_t m, int64_t npix, const float* U, const float* B, const float* x,
                      const float* L, const float* scal, float* Uo, void* stream) {
  if (int rc = unroll_check(ctx, m, npix, {U, B, x, L, scal, Uo})) return rc;
  hipLaunchKernelGGL(k_unroll_ustep, dim3(unroll_wgs((long long)m * npix)), dim3(kUnrollThreads), 0,
                     (hipStream_t)stream, m, (long long)npix, U, B, x, L, scal, Uo);
  return launch_status(ctx, "tomo_unroll_ustep");
}

int tomo_unroll_ustep_grad(tomo_ctx* ctx, int32_t m, int64_t npix, const float* G, const float* PtPG, const float* PG,
                           const float* R, int64_t nsino, const float* U, const float* x, const float* L,
                           const float* scal, float* dU, float* dL, float* dx, float* dscal, int32_t accumulate,
                           void* stream) {
  if (int rc = unroll_check(ctx, m, npix, {G, PtPG, PG, R, U, x, L, scal, dU, dL, dx, dscal})) return rc;
  if (nsino < 1) return ctx->fail(TOMO_EINVAL, "bad sinogram size");
  double* part = unroll_parts(ctx);
  if (!part) return ctx->fail(TOMO_ENOMEM, "workspace");
  hipStream_t s = (hipStream_t)stream;
  const int na = unroll_wgs(npix), nb = unroll_wgs(nsino);
  const int acc = accumulate != 0;
  hipLaunchKernelGGL(k_unroll_ustep_grad, dim3(na), dim3(kUnrollThreads), 0, s, m, (long long)npix, G, PtPG, U, x, L,
                     scal, dU, dL, dx, acc, part);
  hipLaunchKernelGGL(k_unroll_dot, dim3(nb), dim3(kUnrollThreads), 0, s, (long long)nsino, PG, R,
                     part + 3 * kUnrollMaxWgs);
  hipLaunchKernelGGL(k_unroll_finish, dim3(1), dim3(256), 0, s, 0, part, na, part + 3 * kUnrollMaxWgs, nb, scal, dscal,
                     acc);
  return launch_status(ctx, "tomo_unroll_ustep_grad");
}

int tomo_unroll_xseg(tomo_ctx* ctx, int32_t m, int32_t n, const int32_t* owner, const float* U, const float* L,
                     const float* x, const float* scal, float eta2, int32_t e2, float* xo, void* stream) {
  if (int rc = unroll_check(ctx, m, (int64_t)n * n, {owner, U, L, x, scal, xo})) return rc;
  if (e2 < 0) return ctx->fail(TOMO_EINVAL, "E2 < 0");
  hipLaunchKernelGGL(k_unroll_xseg, dim3(unroll_wgs((long long)n * n)), dim3(kUnrollThreads), 0, (hipStream_t)stream,
                     n, owner, U, L, x, scal, eta2, e2, xo);
  return launch_status(ctx, "tomo_unroll_xseg");
}

int tomo_unroll_xseg_grad(tomo_ctx* ctx, int32_t m, int32_t n, const int32_t* owner, const float* G, const float* U,
                          const float* L, const float* x, const float* scal, float eta2, int32_t e2, float* dU,
                          float* dL, float* dx, float* dscal, void* stream) {
  if (int rc = unroll_check(ctx, m, (int64_t)n * n, {owner, G, U, L, x, scal, dU, dL, dx, dscal})) return rc;
  if (e2 < 0) return ctx->fail(TOMO_EINVAL, "E2 < 0");
  double* part = unroll_parts(ctx);
  if (!part) return ctx->fail(TOMO_ENOMEM, "workspace");
  hipStream_t s = (hipStream_t)stream;
  const int na = unroll_wgs((long long)n * n);
  hipLaunchKernelGGL(k_unroll_xseg_grad, dim3(na), dim3(kUnrollThreads), 0, s, m, n, owner, G, U, L, x, scal, eta2, e2,
                     dU, dL, dx, part);
  hipLaunchKernelGGL(k_unroll_finish, dim3(1), dim3(256), 0, s, 1, part, na, part, 0, scal, dscal, 0);
  return launch_status(ctx, "tomo_unroll_xseg_grad");
}

int tomo_unroll_seg_dual_grad(tomo_ctx* ctx, int32_t m, int32_t n, const int32_t* owner, const float* Gx,
                              const float* GL, const float* U, const float* L, const float* x, const float* xs,
                              const float* scal, float eta2, int32_t e2, float* dU, float* dL, float* dx, float* dscal,
                              void* stream) {
  if (int rc = unroll_check(ctx, m, (int64_t)n * n, {owner, Gx, GL, U, L, x, xs, scal, dU, dL, dx, dscal})) return rc;
  if (e2 < 0) return ctx->fail(TOMO_EINVAL, "E2 < 0");
  double* part = unroll_parts(ctx);
  if (!part) return ctx->fail(TOMO_ENOMEM, "workspace");
  hipStream_t s = (hipStream_t)stream;
  const int na = unroll_wgs((long long)n * n);
  hipLaunchKernelGGL(k_unroll_segdual_grad, dim3(na), dim3(kUnrollThreads), 0, s, m, n, owner, Gx, GL, U, L, x, xs,
                     scal, eta2, e2, dU, dL, dx, part);
  hipLaunchKernelGGL(k_unroll_finish, dim3(1), dim3(256), 0, s, 1, part, na, part, 0, scal, dscal, 0);
  return launch_status(ctx, "tomo_unroll_seg_dual_grad");
}

int tomo_unroll_xavg(tomo_ctx* ctx, int32_t m, int64_t npix, const float* U, const float* L, const float* scal,
                     float* xo, void* stream) {
  if (int rc = unroll_check(ctx, m, npix, {U, L, scal, xo})) return rc;
  hipLaunchKernelGGL(k_unroll_xavg, dim3(unroll_wgs(npix)), dim3(kUnrollThreads), 0, (hipStream_t)stream, m,
                     (long long)npix, U, L, scal, xo);
  return launch_status(ctx, "tomo_unroll_xavg");
}

int tomo_unroll_xavg_grad(tomo_ctx* ctx, int32_t m, int64_t npix, const float* G, const float* L, const float* scal,
                          float* dU, float* dL, float* dscal, void* stream) {
  if (int rc = unroll_check(ctx, m, npix, {G, L, scal, dU, dL, dscal})) return rc;
  double* part = unroll_parts(ctx);
  if (!part) return ctx->fail(TOMO_ENOMEM, "workspace");
  hipStream_t s = (hipStream_t)stream;
  const int na = unroll_wgs(npix);
  hipLaunchKernelGGL(k_unroll_xavg_grad, dim3(na), dim3(kUnrollThreads), 0, s, m, (long long)npix, G, L, scal, dU, dL,
                     part);
  hipLaunchKernelGGL(k_unroll_finish, dim3(1), dim3(256), 0, s, 1, part, na, part, 0, scal, dscal, 0);
  return launch_status(ctx, "tomo_unroll_xavg_grad");
}

int tomo_unroll_dual(tomo_ctx* ctx, int32_t m, int64_t npix, const float* L, const float* U, const float* xn,
                     const float* scal, float* Lo, void* stream) {
  if (int rc = unroll_check(ctx, m, npix, {L, U, xn, scal, Lo})) return rc;
  hipLaunchKernelGGL(k_unroll_dual, dim3(unroll_wgs((long long)m * npix)), dim3(kUnrollThreads), 0,
                     (hipStream_t)stream, m, (long long)npix, L, U, xn, scal, Lo);
  return launch_status(ctx, "tomo_unroll_dual");
}

int tomo_unroll_dual_grad(tomo_ctx* ctx, int32_t m, int64_t npix, const float* G, const float* U, const float* xn,
                          const float* scal, float* dL, float* dU, float* dxn, float* dscal, void* stream) {
  if (int rc = unroll_check(ctx, m, npix, {G, U, xn, scal, dL, dU, dxn, dscal})) return rc;
  double* part = unroll_parts(ctx);
  if (!part) return ctx->fail(TOMO_ENOMEM, "workspace");
  hipStream_t s = (hipStream_t)stream;
  const int na = unroll_wgs(npix);
  hipLaunchKernelGGL(k_unroll_dual_grad, dim3(na), dim3(kUnrollThreads), 0, s, m, (long long)npix, G, U, xn, scal, dL,
                     dU, dxn, part);
  hipLaunchKernelGGL(k_unroll_finish, dim3(1), dim3(256), 0, s, 1, part, na, part, 0, scal, dscal, 0);
  return launch_status(ctx, "tomo_unroll_dual_grad");
}

}  // extern "C"
