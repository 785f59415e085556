// Host runtime and C ABI of the MI355X modified Born series solver.
//
// A plan owns, per slot (independent solve): the iterate x, the work array W
// and the diagonal B = 1 - c (k^2 - k_b^2) of (I - V), all subdomain-major
// ([S][n0][n1][n2], z contiguous; W stored slab by slab, with a z-line copy W2 of
// the inverse y pass's output, when the strided passes run on slabs), four
// t-deep edge-slab buffers per corrected axis, the source on its bounding box and
// the FP64 residual partials.  The
// FP64 scalars of Eq. 9 (k_b^2, ||k^2 - k_b^2||_inf, ||A12||, c) live on the
// host.  Iterations are enqueued as hipGraphs of `check_every` iterations over
// all slots; a slot whose device stop flag is set skips every kernel.  Between
// graph launches the host collects finished slots and, for plans with subdomain
// activation, lets idle subdomains join.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mbs.h"
#include "mbs_internal.h"

using namespace mbs;

namespace {

constexpr int kKinds = 9;
enum Kind { kFirst = 0, kMidF = 1, kGreen = 2, kMidI = 3, kLast = 4, kCorr = 5, kFace = 6, kReduce = 7, kSlabs = 8 };

// largest singular value of a small real matrix: sqrt of the largest eigenvalue of
// M^T M by cyclic Jacobi rotations (FP64)
double spectral_norm_jacobi(const std::vector<double>& M, int t) {
  std::vector<double> A(t * t, 0.0);
  for (int i = 0; i < t; ++i)
    for (int j = 0; j < t; ++j) {
      double s = 0.0;
      for (int k = 0; k < t; ++k) s += M[k * t + i] * M[k * t + j];
      A[i * t + j] = s;
    }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < t; ++i)
      for (int j = i + 1; j < t; ++j) off += A[i * t + j] * A[i * t + j];
    if (off < 1e-30) break;
    for (int p = 0; p < t; ++p)
      for (int q = p + 1; q < t; ++q) {
        const double apq = A[p * t + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[p * t + p], aqq = A[q * t + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < t; ++k) {
          const double akp = A[k * t + p], akq = A[k * t + q];
          A[k * t + p] = c * akp - s * akq;
          A[k * t + q] = s * akp + c * akq;
        }
        for (int k = 0; k < t; ++k) {
          const double apk = A[p * t + k], aqk = A[q * t + k];
          A[p * t + k] = c * apk - s * aqk;
          A[q * t + k] = s * apk + c * aqk;
        }
      }
  }
  double mx = 0.0;
  for (int i = 0; i < t; ++i) mx = std::max(mx, A[i * t + i]);
  return std::sqrt(mx);
}

// 1D kernel of the Fourier Laplacian on the infinite unit grid (Sec. 3, Fig. 4):
// l(m) = 2 (-1)^(m+1) / m^2 for m != 0
double lap_kernel(int m) {
  if (m == 0) return -M_PI * M_PI / 3.0;
  const double mm = (double)m;
  return ((std::abs(m) % 2) ? 2.0 : -2.0) / (mm * mm);
}

struct Slot {
  float2* x = nullptr;
  float2* W = nullptr;
  float2* W2 = nullptr;  // z-line output of the inverse y pass when W is blocked; else W
  float2* B = nullptr;
  float2* slab[3][4] = {};
  float2* ybox = nullptr;
  size_t ybox_cap = 0;  // elements
  int ylo[3] = {0, 0, 0}, yext[3] = {0, 0, 0};
  double* part_main = nullptr;
  double* part_face = nullptr;
  double* hist = nullptr;
  double* part_red = nullptr;
  bool has_medium = false;
  bool has_source = false;
  bool busy = false;       // a solve was started and has not been collected
  bool finishing = false;  // result copied out, waiting on `done_ev`
  hipEvent_t done_ev = nullptr;
  void* field_out = nullptr;
  double kb2 = 0, c_im = 0, K = 0;
  bool b_ramp = false;  // lossless medium: B holds Im B only (SlotDesc::b_ramp)
  double k0sq = 0, ramp_max = 0;
  int32_t ramp_w[3] = {0, 0, 0};
  double rho_ref = 0;
  int32_t last_status = MBS_OK;
  int64_t start_seq = 0;   // chunks launched before this solve started
  int64_t launched = 0;    // iterations enqueued since the solve started
  int32_t max_iter = 0;
  mbs_result res{};
  // subdomain activation (Sec. 3.1): bit mask and ascending list of iterated subdomains
  uint32_t* act_d = nullptr;      // device, act_words entries
  int32_t* list_d = nullptr;      // device, S entries
  uint32_t* fresh_d = nullptr;    // device, subdomains activated at the last chunk boundary
  uint32_t* stage = nullptr;      // pinned staging: act words, fresh words, list
  std::vector<uint32_t> act_h;    // host copy of the mask
  int32_t n_act = 0;
  int64_t sub_iters = 0;          // sum over iterations of the subdomains iterated
  int32_t iter_seen = 0;          // iterations accounted in sub_iters (progress of a running solve)
  double eps_seen = 0;            // relative residual of the last iteration seen by the host
};

}  // namespace

struct mbs_plan_s {
  mbs_plan_desc desc{};
  Geo geo{};
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  hipStream_t side_stream = nullptr; // second stream of the slab schedule (every other slab)
  int slab_streams = 1;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int nslots = 0;
  bool corr = false;
  bool fused = false;       // fused z passes (last inverse + next forward)
  bool corr01 = false;     // x or y axis corrected
  double normC = 0;
  int check_every = 16;
  bool use_graph = true;
  bool timing = false;
  int64_t n_main = 0, n_face = 0;
  double activation = 0;    // > 0: subdomain activation with this threshold (relative to rho_ref)
  int zblock = 0;           // > 0: column passes block by block of this many z values
  int act_words = 0;
  double* d_xfer = nullptr;       // nslots x S x kXferBlocks transfer partials
  double* h_xfer = nullptr;       // pinned, 2 x the above
  SlotDesc* d_fresh_tab = nullptr;  // per slot: descriptor that writes W only on fresh subdomains
  // tables
  float2* tw[3] = {};
  float* p2[3] = {};
  float* Cdev = nullptr;
  Tables tb{};
  // slots
  std::vector<Slot> slots;
  std::vector<SlotDesc> h_tab;
  SlotDesc* d_tab = nullptr;       // nslots entries
  SlotDesc* d_probe_tab = nullptr; // 1 entry
  SlotState* d_states = nullptr;   // nslots + 1 (probe)
  SlotState* h_states = nullptr;   // pinned, 2 x (nslots + 1)
  float2* probe_x = nullptr;       // lazily allocated scratch iterate
  int32_t* d_bbox = nullptr;
  int32_t* h_bbox = nullptr;       // pinned
  MediumStats* d_stats = nullptr;
  double* d_kmax = nullptr;
  std::vector<MediumStats> h_stats;
  std::vector<double> h_kmax;
  int64_t setup_nb = 0;
  // graph of check_every iterations over all slots
  hipGraphExec_t graph = nullptr;
  // chunk bookkeeping for asynchronous progress
  bool in_flight = false;
  int64_t chunk_seq = 0;   // number of chunks launched
  hipEvent_t chunk_ev = nullptr;
  int cur_buf = 0;
  // timing
  std::vector<hipEvent_t> tev;  // pairs per launch of one chunk
  std::vector<int> tkind;
  int tcount = 0;
  double t_ms[kKinds] = {};
  int64_t t_launch[kKinds] = {};
  std::vector<void*> allocs;
};

namespace {

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return MBS_EHIP;    \
  } while (0)

bool valid_n(int n) { return n >= 8 && n <= 1024 && fft_size_supported(n); }

// Memory-side cache (Infinity Cache) of the device, in bytes: 256 MB on MI355X.
constexpr size_t kMallBytes = (size_t)256 << 20;
// Slab height of the strided passes and the streams its slabs alternate over.  Automatic: when
// the work arrays of the plan exceed the memory-side cache, whole subdomains on two streams if two
// of them fit in the cache together (one subdomain's passes then overlap the start and the tail
// of the other's); else the largest multiple of 16 dividing n_2 whose slab (n_0 n_1 z complex64
// values of one subdomain) fits in it, on one stream; otherwise every pass runs over every
// subdomain.  A given slab height runs on one stream.
int choose_zblock(const mbs_plan_desc* d, const Geo& g, bool fused, int* streams = nullptr) {
  if (streams) *streams = 1;
  if (!fused || d->zblock < 0) return 0;
  if (d->zblock > 0) return d->zblock;
  const size_t plane = (size_t)g.n[0] * g.n[1] * sizeof(float2);
  if ((size_t)g.S * g.sub_vox * sizeof(float2) * d->max_batch <= kMallBytes) return 0;
  const int wy = col_chunk_width(g.n[1], 0), wx = col_chunk_width(g.n[0], 2);
  auto ok = [&](int z) { return g.n[2] % z == 0 && z % 16 == 0 && z % wy == 0 && z % wx == 0; };
  if (ok(g.n[2]) && plane * g.n[2] * d->max_batch * 2 <= kMallBytes) {
    if (streams) *streams = 2;
    return g.n[2];
  }
  for (int z = g.n[2]; z >= 16; --z)
    if (ok(z) && plane * z * d->max_batch <= kMallBytes) return z;
  return 0;
}

// With the slab schedule, W is stored in blocks of zblock z values when n_2 and zblock are powers
// of two (zblock < n_2), so each slab of the strided passes is one contiguous range of memory;
// otherwise in z-lines.  The arithmetic is the same either way.
void set_w_layout(Geo& g, int zblock) {
  g.wsh = -1;
  g.wplane = 0;
  const int n2 = g.n[2];
  if (zblock <= 0 || zblock >= n2 || (zblock & (zblock - 1)) != 0 || (n2 & (n2 - 1)) != 0) return;
  int sh = 0;
  while ((1 << sh) < zblock) ++sh;
  g.wsh = sh;
  g.wplane = (int64_t)g.n[0] * g.n[1] * zblock;
}

mbs_status validate(const mbs_plan_desc* d, Geo* g) {
  if (!d) return MBS_EINVAL;
  g->wsh = -1;  // W in z-lines unless the slab schedule blocks it (set_w_layout)
  g->wplane = 0;
  if (d->max_batch < 1 || d->max_batch > 4096) return MBS_EINVAL;
  if (!(d->alpha > 0.0 && d->alpha <= 1.0)) return MBS_EINVAL;
  if (d->check_every < 0) return MBS_EINVAL;
  if (!(d->activation >= 0.0 && std::isfinite(d->activation))) return MBS_EINVAL;
  if (d->zblock < -1 || d->reserved != 0) return MBS_EINVAL;
  Geo geo{};
  int64_t sub = 1, vox = 1;
  int S = 1;
  for (int k = 0; k < 3; ++k) {
    if (d->shape[k] < 1 || d->split[k] < 1 || d->shape[k] > (1 << 20)) return MBS_EINVAL;
    if (d->shape[k] % d->split[k] != 0) return MBS_EINVAL;
    const int64_t n = d->shape[k] / d->split[k];
    if (!valid_n((int)n)) return MBS_EUNSUPPORTED;
    geo.n[k] = (int)n;
    geo.P[k] = d->split[k];
    geo.N[k] = (int)d->shape[k];
    geo.periodic[k] = d->periodic[k] ? 1 : 0;
    geo.a[k] = d->split[k] >= 2 ? 2 : (d->periodic[k] ? 0 : 1);
    sub *= n;
    vox *= d->shape[k];
    S *= d->split[k];
  }
  if (vox > (int64_t)1 << 31) return MBS_EUNSUPPORTED;
  const bool corr = geo.a[0] || geo.a[1] || geo.a[2];
  if (corr) {
    if (d->t < 1 || d->t > kMaxT) return MBS_EINVAL;
    for (int k = 0; k < 3; ++k)
      if (geo.a[k] && d->t > geo.n[k] / 2) return MBS_EINVAL;
  }
  geo.t = corr ? d->t : (d->t >= 1 && d->t <= kMaxT ? d->t : 8);
  geo.S = S;
  geo.sub_vox = sub;
  geo.vox = vox;
  geo.face_vox = 0;
  for (int r = 0; r < 3; ++r) {
    geo.reg_count[r] = 0;
    for (int k = 0; k < 3; ++k) {
      if (k == r) {
        geo.reg_ext[r][k] = 2 * geo.t;
        geo.reg_off[r][k] = 0;
      } else if (k < r && geo.a[k]) {
        geo.reg_ext[r][k] = geo.n[k] - 2 * geo.t;
        geo.reg_off[r][k] = geo.t;
      } else {
        geo.reg_ext[r][k] = geo.n[k];
        geo.reg_off[r][k] = 0;
      }
    }
    if (geo.a[r]) {
      geo.reg_count[r] = (int64_t)geo.reg_ext[r][0] * geo.reg_ext[r][1] * geo.reg_ext[r][2];
      geo.face_vox += geo.reg_count[r];
    }
  }
  if (d->zblock > 0) {
    // slabs of the strided passes: whole tiles of both column kinds, fused sequence only
    const int n2 = geo.n[2];
    if (n2 % d->zblock != 0 || d->zblock % col_chunk_width(geo.n[1], 0) != 0 ||
        d->zblock % col_chunk_width(geo.n[0], 2) != 0 || d->zblock % 16 != 0)
      return MBS_EINVAL;
    if ((d->flags & MBS_NO_FUSION) || !fusion_supported(geo)) return MBS_EINVAL;
  }
  if (d->activation > 0.0) {
    // activation skips whole subdomains of the fused z-pass sequence
    if (S > kMaxActSub) return MBS_EUNSUPPORTED;
    if ((d->flags & MBS_NO_FUSION) || !fusion_supported(geo)) return MBS_EUNSUPPORTED;
  }
  *g = geo;
  return MBS_OK;
}

int64_t slab_elems(const Geo& g, int d) {
  const int64_t plane = d == 0 ? (int64_t)g.n[1] * g.n[2]
                               : (d == 1 ? (int64_t)g.n[0] * g.n[2] : (int64_t)g.n[0] * g.n[1]);
  return (int64_t)g.S * 2 * g.t * plane;
}

size_t default_ybox(const Geo& g) {
  const int64_t a = (int64_t)g.N[0] * g.N[1], b = (int64_t)g.N[0] * g.N[2], c = (int64_t)g.N[1] * g.N[2];
  return (size_t)std::max(a, std::max(b, c));
}

size_t slot_bytes(const Geo& g) {
  size_t b = (g.wsh >= 0 ? 4 : 3) * (size_t)g.vox * sizeof(float2);  // x, W, B (and W2)
  for (int d = 0; d < 3; ++d)
    if (g.a[d]) b += 4 * (size_t)slab_elems(g, d) * sizeof(float2);
  b += default_ybox(g) * sizeof(float2);
  b += (size_t)(last_pass_blocks(g) + std::max(face_blocks(g), slabA_blocks(g)) + 1) * sizeof(double);
  b += (size_t)(kHistCap + kReduceBlocks) * sizeof(double);
  return b;
}

template <class T>
mbs_status dalloc(mbs_plan p, T** out, size_t count) {
  void* ptr = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&ptr, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return MBS_ENOMEM;
  }
  p->allocs.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return MBS_OK;
}

void fill_desc(mbs_plan p, int i) {
  Slot& s = p->slots[i];
  SlotDesc& d = p->h_tab[i];
  d.x = s.x;
  d.W = s.W;
  d.W2 = s.W2;
  d.B = s.B;
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 4; ++k) d.slab[a][k] = s.slab[a][k];
  d.ybox = s.ybox;
  for (int k = 0; k < 3; ++k) {
    d.ylo[k] = s.ylo[k];
    d.yext[k] = s.has_source ? s.yext[k] : 0;
  }
  d.c_im = (float)s.c_im;
  d.alpha = (float)p->desc.alpha;
  d.kb2 = (float)s.kb2;
  d.inv_vox = (float)(1.0 / (double)p->geo.sub_vox);
  d.st = p->d_states + i;
  d.part_main = s.part_main;
  d.part_face = s.part_face;
  d.hist = s.hist;
  d.part_red = s.part_red;
  const bool act = p->activation > 0.0 && s.act_d != nullptr;
  d.act = act ? s.act_d : nullptr;
  d.act_list = act ? s.list_d : nullptr;
  d.n_act = act ? s.n_act : p->geo.S;
  d.xfer = act ? p->d_xfer + (size_t)i * p->geo.S * kXferBlocks : nullptr;
  d.b_ramp = s.b_ramp ? 1 : 0;
  d.bx_k = (float)(s.c_im * s.k0sq);
  for (int k = 0; k < 3; ++k) {
    d.rw[k] = s.ramp_w[k];
    d.rstep[k] = s.ramp_w[k] > 0 ? (float)(s.ramp_max / (double)s.ramp_w[k]) : 0.f;
  }
}

mbs_status push_desc(mbs_plan p, int i) {
  fill_desc(p, i);
  HIP_TRY(put_desc(p->d_tab + i, p->h_tab[i], p->stream));
  return MBS_OK;
}

// enqueue one iteration with separate first and last z passes (also used by residual probes)
hipError_t enqueue_iteration_unfused(mbs_plan p, const SlotDesc* tab, int nslots, hipStream_t s) {
  const Geo& g = p->geo;
  auto rec = [&](int kind, bool start) {
    if (!p->timing) return;
    const int idx = p->tcount;
    if (start) {
      if ((size_t)(2 * idx + 1) >= p->tev.size()) {
        const size_t old = p->tev.size();
        p->tev.resize(old + 64);
        p->tkind.resize(p->tev.size() / 2);
        for (size_t k = old; k < p->tev.size(); ++k) (void)hipEventCreate(&p->tev[k]);
      }
      p->tkind[idx] = kind;
      (void)hipEventRecord(p->tev[2 * idx], s);
    } else {
      (void)hipEventRecord(p->tev[2 * idx + 1], s);
      p->tcount++;
    }
  };
  hipError_t e;
  if (p->corr) {
    rec(kCorr, true);
    if ((e = launch_corr(tab, nslots, g, p->tb, 0, s)) != hipSuccess) return e;
    rec(kCorr, false);
  }
  rec(kFirst, true);
  if ((e = launch_first_pass(tab, nslots, g, p->tb, s)) != hipSuccess) return e;
  rec(kFirst, false);
  rec(kMidF, true);
  if ((e = launch_mid_pass(tab, nslots, g, p->tb, 0, s)) != hipSuccess) return e;
  rec(kMidF, false);
  rec(kGreen, true);
  if ((e = launch_green_pass(tab, nslots, g, p->tb, s)) != hipSuccess) return e;
  rec(kGreen, false);
  rec(kMidI, true);
  if ((e = launch_mid_pass(tab, nslots, g, p->tb, 1, s)) != hipSuccess) return e;
  rec(kMidI, false);
  rec(kLast, true);
  if ((e = launch_last_pass(tab, nslots, g, p->tb, s)) != hipSuccess) return e;
  rec(kLast, false);
  if (p->corr) {
    rec(kCorr, true);
    if ((e = launch_corr(tab, nslots, g, p->tb, 1, s)) != hipSuccess) return e;
    rec(kCorr, false);
    rec(kFace, true);
    if ((e = launch_face(tab, nslots, g, s)) != hipSuccess) return e;
    rec(kFace, false);
  }
  rec(kReduce, true);
  if ((e = launch_reduce(tab, nslots, g, p->n_main, p->corr ? p->n_face : 0, s)) != hipSuccess) return e;
  rec(kReduce, false);
  return hipSuccess;
}

// enqueue one iteration with the fused z pass: the forward z FFT of the next iteration is
// produced by the same pass that finishes this one (W must already hold this iteration's
// forward z transform: see start_solve)
hipError_t enqueue_iteration(mbs_plan p, const SlotDesc* tab, int nslots, hipStream_t s) {
  if (!p->fused) return enqueue_iteration_unfused(p, tab, nslots, s);
  const Geo& g = p->geo;
  auto rec = [&](int kind, bool start) {
    if (!p->timing) return;
    const int idx = p->tcount;
    if (start) {
      if ((size_t)(2 * idx + 1) >= p->tev.size()) {
        const size_t old = p->tev.size();
        p->tev.resize(old + 64);
        p->tkind.resize(p->tev.size() / 2);
        for (size_t k = old; k < p->tev.size(); ++k) (void)hipEventCreate(&p->tev[k]);
      }
      p->tkind[idx] = kind;
      (void)hipEventRecord(p->tev[2 * idx], s);
    } else {
      (void)hipEventRecord(p->tev[2 * idx + 1], s);
      p->tcount++;
    }
  };
  hipError_t e;
  if (p->zblock > 0) {
    // the three column passes block by block (one subdomain, zblock z values: a working set
    // that stays in the memory-side cache between the passes)
    // one timing record for the whole slab sequence (events between its many short launches
    // would add gaps of their own)
    const int wy = col_chunk_width(g.n[1], 0), wx = col_chunk_width(g.n[0], 2);
    rec(kSlabs, true);
    // with a side stream, every other slab runs there: the slabs are independent, so one slab's
    // passes overlap the start and the tail of the other's
    const bool two = p->side_stream != nullptr;
    if (two) {
      if ((e = hipEventRecord(p->fork_ev, s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(p->side_stream, p->fork_ev, 0)) != hipSuccess) return e;
    }
    int k = 0;
    for (int sub = 0; sub < g.S; ++sub)
      for (int z0 = 0; z0 < g.n[2]; z0 += p->zblock, ++k) {
        const ColRange ry{sub, 1, z0 / wy, p->zblock / wy}, rx{sub, 1, z0 / wx, p->zblock / wx};
        hipStream_t st = (two && (k & 1)) ? p->side_stream : s;
        if ((e = launch_mid_pass(tab, nslots, g, p->tb, 0, st, ry)) != hipSuccess) return e;
        if ((e = launch_green_pass(tab, nslots, g, p->tb, st, rx)) != hipSuccess) return e;
        if ((e = launch_mid_pass(tab, nslots, g, p->tb, 1, st, ry)) != hipSuccess) return e;
      }
    if (two) {
      if ((e = hipEventRecord(p->join_ev, p->side_stream)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(s, p->join_ev, 0)) != hipSuccess) return e;
    }
    rec(kSlabs, false);
  } else {
    rec(kMidF, true);
    if ((e = launch_mid_pass(tab, nslots, g, p->tb, 0, s)) != hipSuccess) return e;
    rec(kMidF, false);
    rec(kGreen, true);
    if ((e = launch_green_pass(tab, nslots, g, p->tb, s)) != hipSuccess) return e;
    rec(kGreen, false);
    rec(kMidI, true);
    if ((e = launch_mid_pass(tab, nslots, g, p->tb, 1, s)) != hipSuccess) return e;
    rec(kMidI, false);
  }
  rec(kLast, true);
  if ((e = launch_fused(tab, nslots, g, p->tb, s)) != hipSuccess) return e;
  rec(kLast, false);
  if (p->corr01) {
    rec(kCorr, true);
    if ((e = launch_corr(tab, nslots, g, p->tb, 1, s, 3)) != hipSuccess) return e;
    rec(kCorr, false);
    rec(kFace, true);
    if ((e = launch_slabA(tab, nslots, g, s)) != hipSuccess) return e;
    rec(kFace, false);
    rec(kCorr, true);
    if ((e = launch_corr(tab, nslots, g, p->tb, 0, s, 3)) != hipSuccess) return e;
    rec(kCorr, false);
    rec(kFirst, true);
    if ((e = launch_wpass(tab, nslots, g, p->tb, 1, s)) != hipSuccess) return e;
    rec(kFirst, false);
  }
  rec(kReduce, true);
  if ((e = launch_reduce(tab, nslots, g, p->n_main, p->corr01 ? slabA_blocks(g) : 0, s)) != hipSuccess) return e;
  rec(kReduce, false);
  return hipSuccess;
}

mbs_status build_graph(mbs_plan p) {
  if (p->graph) return MBS_OK;
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int it = 0; it < p->check_every && e == hipSuccess; ++it)
    e = enqueue_iteration(p, p->d_tab, p->nslots, p->cap_stream);
  if (e == hipSuccess && p->activation > 0.0) e = launch_xfer(p->d_tab, p->nslots, p->geo, p->tb, p->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return MBS_EHIP;
  }
  hipError_t e3 = hipGraphInstantiate(&p->graph, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e3 != hipSuccess) {
    p->graph = nullptr;
    return MBS_EHIP;
  }
  return MBS_OK;
}

// enqueue check_every iterations for all slots, then copy the slot states to the host
mbs_status launch_chunk(mbs_plan p) {
  int64_t n_it = p->check_every;
  if (p->use_graph) {
    mbs_status st = build_graph(p);
    if (st != MBS_OK) return st;
    HIP_TRY(hipGraphLaunch(p->graph, p->stream));
  } else {
    // eager launches: no more iterations than the running slots can still use
    int64_t need = 0;
    for (auto& s : p->slots)
      if (s.busy && !s.finishing) need = std::max(need, (int64_t)s.max_iter - s.launched);
    n_it = std::max<int64_t>(1, std::min<int64_t>(p->check_every, need));
    p->tcount = 0;
    for (int64_t it = 0; it < n_it; ++it)
      HIP_TRY(enqueue_iteration(p, p->d_tab, p->nslots, p->stream));
    if (p->activation > 0.0) HIP_TRY(launch_xfer(p->d_tab, p->nslots, p->geo, p->tb, p->stream));
  }
  for (auto& s : p->slots)
    if (s.busy && !s.finishing) s.launched += n_it;
  p->cur_buf ^= 1;
  SlotState* hb = p->h_states + p->cur_buf * (p->nslots + 1);
  HIP_TRY(hipMemcpyAsync(hb, p->d_states, sizeof(SlotState) * p->nslots, hipMemcpyDeviceToHost, p->stream));
  if (p->activation > 0.0) {
    const size_t nx = (size_t)p->nslots * p->geo.S * kXferBlocks;
    HIP_TRY(hipMemcpyAsync(p->h_xfer + p->cur_buf * nx, p->d_xfer, nx * sizeof(double), hipMemcpyDeviceToHost,
                           p->stream));
  }
  HIP_TRY(hipEventRecord(p->chunk_ev, p->stream));
  p->in_flight = true;
  p->chunk_seq++;
  return MBS_OK;
}

void collect_timing(mbs_plan p) {
  if (!p->timing) return;
  for (int i = 0; i < p->tcount; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->tev[2 * i], p->tev[2 * i + 1]) == hipSuccess) {
      p->t_ms[p->tkind[i]] += ms;
      p->t_launch[p->tkind[i]] += 1;
    }
  }
  p->tcount = 0;
}

int32_t status_of(int32_t done) {
  switch (done) {
    case kDiverged: return MBS_EDIVERGED;
    case kNonFinite: return MBS_ENONFINITE;
    default: return MBS_OK;
  }
}

// finish slots whose device state says done: copy the field out, mark idle on the device
mbs_status retire_finished(mbs_plan p, const SlotState* hs) {
  for (int i = 0; i < p->nslots; ++i) {
    Slot& s = p->slots[i];
    if (!s.busy || s.finishing) continue;
    if (p->chunk_seq <= s.start_seq) continue;  // that chunk was launched before the solve started
    const SlotState& st = hs[i];
    if (st.done == kRunning) continue;
    mbs_result& r = s.res;
    r.iterations = st.iter;
    r.rel_residual = st.eps;
    r.converged = st.done == kConverged ? 1 : 0;
    r.kb2 = s.kb2;
    r.c_imag = s.c_im;
    r.K = s.K;
    r.normC = p->normC;
    r.rho_ref = st.rho_ref;
    r.status = status_of(st.done);
    r.subdomain_iterations = s.sub_iters;
    s.rho_ref = st.rho_ref;
    s.last_status = r.status;
    if (s.field_out) HIP_TRY(launch_gather(s.x, p->geo, (float2*)s.field_out, p->stream));
    HIP_TRY(hipEventRecord(s.done_ev, p->stream));
    s.finishing = true;
  }
  return MBS_OK;
}

// copy a slot's activation mask, its list of iterated subdomains and (optionally) the mask of
// newly activated subdomains to the device, through the slot's pinned staging buffer
mbs_status upload_activation(mbs_plan p, int i, const std::vector<uint32_t>* fresh) {
  Slot& s = p->slots[i];
  const int S = p->geo.S, W = p->act_words;
  uint32_t* stg = s.stage;  // [W mask][W fresh][S list]
  int32_t* list = reinterpret_cast<int32_t*>(stg + 2 * W);
  std::copy(s.act_h.begin(), s.act_h.end(), stg);
  int n = 0;
  for (int sub = 0; sub < S; ++sub)
    if ((s.act_h[sub >> 5] >> (sub & 31)) & 1u) list[n++] = sub;
  s.n_act = n;
  HIP_TRY(hipMemcpyAsync(s.act_d, stg, W * sizeof(uint32_t), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(s.list_d, list, S * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  if (fresh) {
    std::copy(fresh->begin(), fresh->end(), stg + W);
    HIP_TRY(hipMemcpyAsync(s.fresh_d, stg + W, W * sizeof(uint32_t), hipMemcpyHostToDevice, p->stream));
  }
  return MBS_OK;
}

// Subdomain activation (Sec. 3.1, end), at a chunk boundary: a subdomain that is not iterated
// joins when the field its iterated neighbours transfer into it (2-norm of the edge terms, from
// k_xfer at the end of the chunk) exceeds activation * rho_ref.  Its w is formed at once (x is
// still zero there), the divergence test is reset for one iteration (the residual grows by the
// new subdomain's share), and a slot that had converged on the old set iterates on.
mbs_status apply_activation(mbs_plan p, SlotState* hs, const double* hx) {
  const int S = p->geo.S, W = p->act_words;
  for (int i = 0; i < p->nslots; ++i) {
    Slot& s = p->slots[i];
    if (!s.busy || s.finishing || p->chunk_seq <= s.start_seq) continue;
    SlotState& st = hs[i];
    if (st.done != kRunning && st.done != kConverged) continue;
    if (!(st.rho_ref > 0.0)) continue;
    const double thr = p->activation * st.rho_ref;
    std::vector<uint32_t> fresh(W, 0u);
    bool any = false;
    for (int sub = 0; sub < S; ++sub) {
      if ((s.act_h[sub >> 5] >> (sub & 31)) & 1u) continue;
      const double* part = hx + ((size_t)i * S + sub) * kXferBlocks;
      double sum = 0.0;
      for (int b = 0; b < kXferBlocks; ++b) sum += part[b];
      if (sum > thr * thr) {
        fresh[sub >> 5] |= 1u << (sub & 31);
        any = true;
      }
    }
    if (!any) continue;
    for (int w = 0; w < W; ++w) s.act_h[w] |= fresh[w];
    mbs_status r = upload_activation(p, i, &fresh);
    if (r != MBS_OK) return r;
    r = push_desc(p, i);
    if (r != MBS_OK) return r;
    SlotDesc fd = p->h_tab[i];
    fd.act = s.fresh_d;  // write W on the fresh subdomains only
    fd.act_list = nullptr;
    fd.xfer = nullptr;
    HIP_TRY(put_desc(p->d_fresh_tab + i, fd, p->stream));
    SlotState ns = st;
    ns.done = kRunning;
    ns.eps_prev = HUGE_VAL;
    HIP_TRY(put_state(p->d_states + i, ns, p->stream));
    HIP_TRY(launch_wpass(p->d_fresh_tab + i, 1, p->geo, p->tb, 0, p->stream));
    st.done = kRunning;  // not finished after all
  }
  return MBS_OK;
}

// initial set of iterated subdomains: those holding source (all of them with a given start
// field or without a source)
mbs_status init_activation(mbs_plan p, int i, bool all) {
  Slot& s = p->slots[i];
  const Geo& g = p->geo;
  s.act_h.assign(p->act_words, 0u);
  for (int sub = 0; sub < g.S; ++sub) {
    const int sc[3] = {sub / (g.P[1] * g.P[2]), (sub / g.P[2]) % g.P[1], sub % g.P[2]};
    bool on = true;
    if (!all)
      for (int k = 0; k < 3; ++k) {
        const int lo = sc[k] * g.n[k], hi = lo + g.n[k];
        if (s.ylo[k] >= hi || s.ylo[k] + s.yext[k] <= lo) on = false;
      }
    if (on) s.act_h[sub >> 5] |= 1u << (sub & 31);
  }
  mbs_status r = upload_activation(p, i, nullptr);
  if (r != MBS_OK) return r;
  // u of subdomains that are not iterated is zero; their edge values must read as zero
  for (int d = 0; d < 2; ++d)
    if (g.a[d]) HIP_TRY(launch_zero(s.slab[d][1], slab_elems(g, d), p->stream));
  return MBS_OK;
}

bool any_running(mbs_plan p) {
  for (auto& s : p->slots)
    if (s.busy && !s.finishing) return true;
  return false;
}

// advance the plan without blocking (or blocking until the in-flight chunk ends)
mbs_status progress(mbs_plan p, bool block) {
  if (p->in_flight) {
    if (block) {
      HIP_TRY(hipEventSynchronize(p->chunk_ev));
    } else {
      hipError_t q = hipEventQuery(p->chunk_ev);
      if (q == hipErrorNotReady) return MBS_OK;
      if (q != hipSuccess) return MBS_EHIP;
    }
    p->in_flight = false;
    collect_timing(p);
    SlotState* hs = p->h_states + p->cur_buf * (p->nslots + 1);
    mbs_status st = MBS_OK;
    for (int i = 0; i < p->nslots; ++i) {  // subdomain-iterations of the chunk, on the set it ran with
      Slot& s = p->slots[i];
      if (!s.busy || s.finishing || p->chunk_seq <= s.start_seq) continue;
      const int32_t n_set = p->activation > 0.0 ? s.n_act : p->geo.S;
      s.sub_iters += (int64_t)(hs[i].iter - s.iter_seen) * n_set;
      s.iter_seen = hs[i].iter;
      s.eps_seen = hs[i].eps;
    }
    if (p->activation > 0.0) {
      const size_t nx = (size_t)p->nslots * p->geo.S * kXferBlocks;
      st = apply_activation(p, hs, p->h_xfer + p->cur_buf * nx);
      if (st != MBS_OK) return st;
    }
    st = retire_finished(p, hs);
    if (st != MBS_OK) return st;
  }
  if (any_running(p)) return launch_chunk(p);
  return MBS_OK;
}

mbs_status prepare_source(mbs_plan p, int slot, const void* src) {
  Slot& s = p->slots[slot];
  const Geo& g = p->geo;
  const int32_t init[8] = {INT_MAX, INT_MAX, INT_MAX, -1, -1, -1, 0, 0};
  HIP_TRY(put_i32x8(p->d_bbox, init, p->stream));
  HIP_TRY(launch_source_bbox((const float2*)src, g, p->d_bbox, p->stream));
  HIP_TRY(hipMemcpyAsync(p->h_bbox, p->d_bbox, sizeof(init), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (p->h_bbox[6]) return MBS_ENONFINITE;
  if (p->h_bbox[3] < 0) {
    s.has_source = false;
    for (int k = 0; k < 3; ++k) s.yext[k] = 0;
    return MBS_OK;
  }
  size_t cnt = 1;
  for (int k = 0; k < 3; ++k) {
    s.ylo[k] = p->h_bbox[k];
    s.yext[k] = p->h_bbox[3 + k] - p->h_bbox[k] + 1;
    cnt *= (size_t)s.yext[k];
  }
  if (cnt > s.ybox_cap) {
    void* np = nullptr;
    if (hipMalloc(&np, cnt * sizeof(float2)) != hipSuccess) {
      (void)hipGetLastError();
      return MBS_ENOMEM;
    }
    if (s.ybox) {
      HIP_TRY(hipStreamSynchronize(p->stream));
      for (auto& a : p->allocs)
        if (a == s.ybox) a = nullptr;
      (void)hipFree(s.ybox);
    }
    p->allocs.push_back(np);
    s.ybox = (float2*)np;
    s.ybox_cap = cnt;
  }
  HIP_TRY(launch_source_fill((const float2*)src, g, s.ylo, s.yext, s.c_im, s.ybox, p->stream));
  s.has_source = true;
  return MBS_OK;
}

// one evaluation of d = (I-V)(x - (L+I)^-1 [y + (I-V) x]) without updating x; returns ||d||
mbs_status probe_norm(mbs_plan p, int slot, float2* xsrc, double* rho) {
  Slot& s = p->slots[slot];
  fill_desc(p, slot);
  SlotDesc d = p->h_tab[slot];
  d.x = xsrc;
  d.alpha = 0.f;
  d.st = p->d_states + p->nslots;
  d.act = nullptr;  // a residual evaluation covers every subdomain
  d.act_list = nullptr;
  d.n_act = p->geo.S;
  d.xfer = nullptr;
  SlotState st{};
  st.done = kRunning;
  st.probe = 1;
  st.max_iter = 1;
  st.tol = 0;
  HIP_TRY(put_desc(p->d_probe_tab, d, p->stream));
  HIP_TRY(put_state(p->d_states + p->nslots, st, p->stream));
  if (p->corr && xsrc != s.x) {
    HIP_TRY(launch_extract_slabs(p->d_probe_tab, 0, p->geo, 0, p->stream));
  }
  HIP_TRY(enqueue_iteration_unfused(p, p->d_probe_tab, 1, p->stream));
  SlotState* hb = p->h_states + 2 * (p->nslots + 1) - 1;
  HIP_TRY(hipMemcpyAsync(hb, p->d_states + p->nslots, sizeof(SlotState), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->tcount = 0;
  if (p->corr && xsrc != s.x) {
    // restore the slot's own edge slabs of its iterate
    HIP_TRY(launch_extract_slabs(p->d_tab, slot, p->geo, 0, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  if (hb->done != kConverged) return MBS_ENONFINITE;
  *rho = hb->rho;
  return MBS_OK;
}

mbs_status ensure_probe_x(mbs_plan p) {
  if (p->probe_x) return MBS_OK;
  return dalloc(p, &p->probe_x, (size_t)p->geo.vox);
}

mbs_status start_solve(mbs_plan p, int slot, const void* src, double tol, int32_t max_iter,
                       void* field) {
  if (!p || slot < 0 || slot >= p->nslots || !src) return MBS_EINVAL;
  if (!(tol >= 0.0) || max_iter < 1) return MBS_EINVAL;
  Slot& s = p->slots[slot];
  if (!s.has_medium || s.busy) return MBS_ESTATE;
  const bool x0 = (p->desc.flags & MBS_X0_GIVEN) != 0;
  if (x0 && !field) return MBS_EINVAL;
  mbs_status st = prepare_source(p, slot, src);
  if (st != MBS_OK) return st;
  if (p->activation > 0.0) {
    st = init_activation(p, slot, x0 || !s.has_source);
    if (st != MBS_OK) return st;
  }
  if (x0) HIP_TRY(launch_scatter((const float2*)field, p->geo, s.x, p->stream));
  else HIP_TRY(launch_zero(s.x, p->geo.vox, p->stream));
  st = push_desc(p, slot);
  if (st != MBS_OK) return st;
  if (p->corr) HIP_TRY(launch_extract_slabs(p->d_tab, slot, p->geo, 0, p->stream));
  double rho_ref = 0.0;
  if (x0) {
    // ||Gamma^-1 y|| = ||d|| of the zero field
    st = ensure_probe_x(p);
    if (st != MBS_OK) return st;
    HIP_TRY(launch_zero(p->probe_x, p->geo.vox, p->stream));
    st = probe_norm(p, slot, p->probe_x, &rho_ref);
    if (st != MBS_OK) return st;
  }
  SlotState init{};
  init.rho_ref = rho_ref;
  init.tol = tol;
  init.iter = 0;
  init.max_iter = max_iter;
  init.done = kRunning;
  init.probe = 0;
  HIP_TRY(put_state(p->d_states + slot, init, p->stream));
  if (p->fused) {
    // W of iteration 0 (forward z transform of w_0) for this slot only
    const SlotDesc* one = p->d_tab + slot;
    if (p->corr01) HIP_TRY(launch_corr(one, 1, p->geo, p->tb, 0, p->stream, 3));
    HIP_TRY(launch_wpass(one, 1, p->geo, p->tb, 0, p->stream));
  }
  s.busy = true;
  s.sub_iters = 0;
  s.iter_seen = 0;
  s.eps_seen = 0;
  s.start_seq = p->chunk_seq;
  s.finishing = false;
  s.field_out = field;
  return MBS_OK;
}

mbs_status finish_poll(mbs_plan p, int slot, mbs_result* res) {
  Slot& s = p->slots[slot];
  if (!s.busy) return MBS_ESTATE;
  if (!s.finishing) return MBS_EBUSY;
  hipError_t q = hipEventQuery(s.done_ev);
  if (q == hipErrorNotReady) return MBS_EBUSY;
  if (q != hipSuccess) return MBS_EHIP;
  s.busy = false;
  s.finishing = false;
  // mark idle on the device so batched launches skip the slot
  SlotState idle{};
  idle.done = kIdle;
  idle.rho_ref = s.rho_ref;
  idle.iter = s.res.iterations;
  idle.eps = s.res.rel_residual;
  HIP_TRY(put_state(p->d_states + slot, idle, p->stream));
  if (res) *res = s.res;
  return s.res.status;
}

}  // namespace

extern "C" {

const char* mbs_strerror(mbs_status st) {
  switch (st) {
    case MBS_OK: return "ok";
    case MBS_EINVAL: return "invalid argument";
    case MBS_ENOMEM: return "device out of memory";
    case MBS_EGAIN: return "gain medium: Im k^2 < 0";
    case MBS_EDEGENERATE: return "degenerate scaling: ||k^2-k_b^2|| + sum a_d ||A12|| = 0";
    case MBS_ENONFINITE: return "non-finite value in medium, source or residual";
    case MBS_EDIVERGED: return "residual increased: iteration diverged";
    case MBS_ESTATE: return "invalid slot state (no medium set, or slot busy)";
    case MBS_EBUSY: return "solve still running";
    case MBS_EHIP: return "HIP runtime error";
    case MBS_EUNSUPPORTED: return "unsupported subdomain size";
    default: return "unknown status";
  }
}

mbs_status mbs_plan_bytes(const mbs_plan_desc* desc, size_t* device_bytes) {
  if (!device_bytes) return MBS_EINVAL;
  Geo g{};
  mbs_status st = validate(desc, &g);
  if (st != MBS_OK) return st;
  // the layout of W the plan will choose (plan_create)
  set_w_layout(g, choose_zblock(desc, g, !(desc->flags & MBS_NO_FUSION) && fusion_supported(g)));
  size_t b = (size_t)desc->max_batch * slot_bytes(g);
  b += (size_t)(desc->max_batch + 1) * (sizeof(SlotDesc) + sizeof(SlotState)) + sizeof(SlotDesc);
  for (int d = 0; d < 3; ++d) b += (size_t)g.n[d] * (sizeof(float2) + sizeof(float));
  b += (size_t)kMaxT * kMaxT * sizeof(float);
  b += (size_t)setup_blocks(g) * (sizeof(MediumStats) + sizeof(double)) + 64;
  if (desc->activation > 0.0)  // masks, lists, transfer partials, fresh descriptors
    b += (size_t)desc->max_batch * ((2 * (size_t)((g.S + 31) / 32) + g.S) * sizeof(uint32_t) +
                                    (size_t)g.S * kXferBlocks * sizeof(double) + sizeof(SlotDesc));
  *device_bytes = b;
  return MBS_OK;
}

mbs_status mbs_plan_destroy(mbs_plan p) {
  if (!p) return MBS_EINVAL;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->join_ev) (void)hipEventDestroy(p->join_ev);
  if (p->chunk_ev) (void)hipEventDestroy(p->chunk_ev);
  for (auto& s : p->slots)
    if (s.done_ev) (void)hipEventDestroy(s.done_ev);
  for (auto e : p->tev) (void)hipEventDestroy(e);
  for (void* a : p->allocs)
    if (a) (void)hipFree(a);
  if (p->h_states) (void)hipHostFree(p->h_states);
  if (p->h_xfer) (void)hipHostFree(p->h_xfer);
  for (auto& s : p->slots)
    if (s.stage) (void)hipHostFree(s.stage);
  if (p->h_bbox) (void)hipHostFree(p->h_bbox);
  delete p;
  return MBS_OK;
}

mbs_status mbs_plan_create(const mbs_plan_desc* desc, void* hip_stream, mbs_plan* out) {
  if (!out) return MBS_EINVAL;
  *out = nullptr;
  Geo g{};
  mbs_status st = validate(desc, &g);
  if (st != MBS_OK) return st;
  mbs_plan p = new (std::nothrow) mbs_plan_s();
  if (!p) return MBS_ENOMEM;
  p->desc = *desc;
  p->geo = g;
  p->stream = (hipStream_t)hip_stream;
  p->nslots = desc->max_batch;
  p->corr = g.a[0] || g.a[1] || g.a[2];
  p->corr01 = g.a[0] || g.a[1];
  p->fused = !(desc->flags & MBS_NO_FUSION) && fusion_supported(g);
  p->activation = desc->activation;
  p->zblock = choose_zblock(desc, g, p->fused, &p->slab_streams);
  set_w_layout(p->geo, p->zblock);
  p->check_every = desc->check_every > 0 ? desc->check_every : 16;
  p->timing = (desc->flags & MBS_TIMING) != 0;
  p->use_graph = !(desc->flags & (MBS_NO_GRAPH | MBS_TIMING));
  p->n_main = last_pass_blocks(g);
  p->n_face = face_blocks(g);
  const int64_t n_part_face = std::max(p->n_face, slabA_blocks(g));  // face or edge-slab partials
  auto fail = [&](mbs_status s) {
    mbs_plan_destroy(p);
    return s;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return fail(MBS_EHIP);
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) return fail(MBS_EHIP);
    p->geo.cus = cus;
  }
  prepare_launches(p->geo);
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) return fail(MBS_EHIP);
  if (p->zblock > 0 && p->slab_streams > 1) {
    if (hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking) != hipSuccess) return fail(MBS_EHIP);
    if (hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) != hipSuccess) return fail(MBS_EHIP);
    if (hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming) != hipSuccess) return fail(MBS_EHIP);
  }
  if (hipEventCreateWithFlags(&p->chunk_ev, hipEventDisableTiming) != hipSuccess) return fail(MBS_EHIP);
  // tables: twiddles, |p|^2 per axis, correction block (FP64 on the host, rounded once)
  for (int d = 0; d < 3; ++d) {
    const int n = g.n[d];
    std::vector<float2> tw(n);
    std::vector<float> p2(n);
    for (int q = 0; q < n; ++q) {
      const double ang = -2.0 * M_PI * (double)q / (double)n;
      tw[q] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      const int qq = q < (n + 1) / 2 ? q : q - n;  // Nyquist of even n at -pi
      const double pp = 2.0 * M_PI * (double)qq / (double)n;
      p2[q] = (float)(pp * pp);
    }
    if ((st = dalloc(p, &p->tw[d], n)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &p->p2[d], n)) != MBS_OK) return fail(st);
    if (hipMemcpy(p->tw[d], tw.data(), n * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return fail(MBS_EHIP);
    if (hipMemcpy(p->p2[d], p2.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return fail(MBS_EHIP);
    p->tb.tw[d] = p->tw[d];
    p->tb.p2[d] = p->p2[d];
  }
  {
    const int t = g.t;
    std::vector<double> C(t * t);
    std::vector<float> Cf(t * t);
    for (int a = 0; a < t; ++a)
      for (int b = 0; b < t; ++b) {
        C[a * t + b] = lap_kernel(a + t - b);  // C[a,b] = l(a + t - b)
        Cf[a * t + b] = (float)C[a * t + b];
      }
    p->normC = spectral_norm_jacobi(C, t);
    if ((st = dalloc(p, &p->Cdev, t * t)) != MBS_OK) return fail(st);
    if (hipMemcpy(p->Cdev, Cf.data(), t * t * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return fail(MBS_EHIP);
    p->tb.C = p->Cdev;
  }
  // slots
  p->slots.resize(p->nslots);
  p->h_tab.resize(p->nslots);
  for (int i = 0; i < p->nslots; ++i) {
    Slot& s = p->slots[i];
    if ((st = dalloc(p, &s.x, g.vox)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &s.W, g.vox)) != MBS_OK) return fail(st);
    s.W2 = s.W;
    if (p->geo.wsh >= 0 && (st = dalloc(p, &s.W2, g.vox)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &s.B, g.vox)) != MBS_OK) return fail(st);
    for (int d = 0; d < 3; ++d)
      if (g.a[d])
        for (int k = 0; k < 4; ++k)
          if ((st = dalloc(p, &s.slab[d][k], slab_elems(g, d))) != MBS_OK) return fail(st);
    s.ybox_cap = default_ybox(g);
    if ((st = dalloc(p, &s.ybox, s.ybox_cap)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &s.part_main, p->n_main)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &s.part_face, n_part_face)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &s.hist, kHistCap)) != MBS_OK) return fail(st);
    if ((st = dalloc(p, &s.part_red, kReduceBlocks)) != MBS_OK) return fail(st);
    if (hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming) != hipSuccess) return fail(MBS_EHIP);
  }
  if (p->activation > 0.0) {
    const int S = g.S, W = (S + 31) / 32;
    p->act_words = W;
    for (int i = 0; i < p->nslots; ++i) {
      Slot& s = p->slots[i];
      if ((st = dalloc(p, &s.act_d, W)) != MBS_OK) return fail(st);
      if ((st = dalloc(p, &s.fresh_d, W)) != MBS_OK) return fail(st);
      if ((st = dalloc(p, &s.list_d, S)) != MBS_OK) return fail(st);
      if (hipHostMalloc((void**)&s.stage, (2 * (size_t)W + S) * sizeof(uint32_t), 0) != hipSuccess)
        return fail(MBS_ENOMEM);
      s.act_h.assign(W, ~0u);
      s.n_act = S;
    }
    const size_t nx = (size_t)p->nslots * S * kXferBlocks;
    if ((st = dalloc(p, &p->d_xfer, nx)) != MBS_OK) return fail(st);
    if (hipHostMalloc((void**)&p->h_xfer, 2 * nx * sizeof(double), 0) != hipSuccess) return fail(MBS_ENOMEM);
    if ((st = dalloc(p, &p->d_fresh_tab, p->nslots)) != MBS_OK) return fail(st);
  }
  if ((st = dalloc(p, &p->d_tab, p->nslots)) != MBS_OK) return fail(st);
  if ((st = dalloc(p, &p->d_probe_tab, 1)) != MBS_OK) return fail(st);
  if ((st = dalloc(p, &p->d_states, p->nslots + 1)) != MBS_OK) return fail(st);
  if (hipHostMalloc((void**)&p->h_states, 2 * (p->nslots + 1) * sizeof(SlotState), 0) != hipSuccess) return fail(MBS_ENOMEM);
  if (hipHostMalloc((void**)&p->h_bbox, 8 * sizeof(int32_t), 0) != hipSuccess) return fail(MBS_ENOMEM);
  if ((st = dalloc(p, &p->d_bbox, 8)) != MBS_OK) return fail(st);
  p->setup_nb = setup_blocks(g);
  if ((st = dalloc(p, &p->d_stats, p->setup_nb)) != MBS_OK) return fail(st);
  if ((st = dalloc(p, &p->d_kmax, p->setup_nb)) != MBS_OK) return fail(st);
  p->h_stats.resize(p->setup_nb);
  p->h_kmax.resize(p->setup_nb);
  // every slot starts idle
  std::vector<SlotState> idle(p->nslots + 1);
  for (auto& s : idle) s.done = kIdle;
  if (hipMemcpy(p->d_states, idle.data(), idle.size() * sizeof(SlotState), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MBS_EHIP);
  for (int i = 0; i < p->nslots; ++i) fill_desc(p, i);
  if (hipMemcpy(p->d_tab, p->h_tab.data(), p->nslots * sizeof(SlotDesc), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MBS_EHIP);
  *out = p;
  return MBS_OK;
}

mbs_status mbs_set_medium(mbs_plan p, int32_t slot, const void* n_dev, double k0, const mbs_ramp* ramp) {
  if (!p || slot < 0 || slot >= p->nslots || !n_dev) return MBS_EINVAL;
  if (!(std::isfinite(k0) && k0 > 0.0)) return MBS_EINVAL;
  Slot& s = p->slots[slot];
  if (s.busy) return MBS_ESTATE;
  int32_t width[3] = {0, 0, 0};
  double rmax = 0.0;
  if (ramp) {
    for (int k = 0; k < 3; ++k) {
      if (ramp->width[k] < 0 || ramp->width[k] > p->geo.N[k]) return MBS_EINVAL;
      width[k] = ramp->width[k];
    }
    if (!std::isfinite(ramp->im_n2_max)) return MBS_EINVAL;
    rmax = ramp->im_n2_max;
  }
  const double k0sq = k0 * k0;
  const Geo& g = p->geo;
  const float2* n = (const float2*)n_dev;
  HIP_TRY(launch_medium_stats(n, g, k0sq, width, rmax, p->d_stats, p->setup_nb, p->stream));
  HIP_TRY(hipMemcpyAsync(p->h_stats.data(), p->d_stats, p->setup_nb * sizeof(MediumStats),
                         hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double re_min = INFINITY, re_max = -INFINITY, im_min = INFINITY, nf = 0, nim_max = 0;
  for (const auto& m : p->h_stats) {
    re_min = std::min(re_min, m.re_min);
    re_max = std::max(re_max, m.re_max);
    im_min = std::min(im_min, m.im_min);
    nf += m.nonfinite;
    nim_max = std::max(nim_max, m.nim_max);
  }
  s.has_medium = false;
  if (nf > 0) return MBS_ENONFINITE;
  if (im_min < 0.0) return MBS_EGAIN;
  const double kb2 = (p->desc.flags & MBS_KB_FROM_K0) ? k0sq : 0.5 * (re_min + re_max);
  HIP_TRY(launch_medium_kmax(n, g, k0sq, width, rmax, kb2, p->d_kmax, p->setup_nb, p->stream));
  HIP_TRY(hipMemcpyAsync(p->h_kmax.data(), p->d_kmax, p->setup_nb * sizeof(double), hipMemcpyDeviceToHost,
                         p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double K = 0.0;
  for (double v : p->h_kmax) K = std::max(K, v);
  // Eq. 9: c = -0.95 i / (||k^2 - k_b^2||_inf + sum_d a_d ||A12||)
  const double denom = K + (double)(g.a[0] + g.a[1] + g.a[2]) * p->normC;
  if (!(denom > 0.0)) return MBS_EDEGENERATE;
  const double c_im = -0.95 / denom;
  // a lossless medium (Im n = 0): Im k^2 is the absorbing ramp alone, so Re B = 1 + c_im k0^2 ramp
  // is a function of position and only Im B is stored
#ifndef MBS_COMPACT_B
#define MBS_COMPACT_B 1
#endif
  const bool compact = MBS_COMPACT_B && nim_max == 0.0;
  HIP_TRY(launch_medium_B(n, g, k0sq, width, rmax, kb2, c_im, s.B, compact ? 1 : 0, p->stream));
  s.b_ramp = compact;
  s.k0sq = k0sq;
  s.ramp_max = rmax;
  for (int k = 0; k < 3; ++k) s.ramp_w[k] = width[k];
  s.kb2 = kb2;
  s.K = K;
  s.c_im = c_im;
  s.has_medium = true;
  s.has_source = false;
  s.rho_ref = 0.0;
  mbs_status st = push_desc(p, slot);
  if (st != MBS_OK) return st;
  HIP_TRY(hipStreamSynchronize(p->stream));
  return MBS_OK;
}

mbs_status mbs_solve_async(mbs_plan p, int32_t slot, const void* src_dev, double tol, int32_t max_iter,
                           void* field_dev) {
  mbs_status st = start_solve(p, slot, src_dev, tol, max_iter, field_dev);
  if (st != MBS_OK) return st;
  if (!p->in_flight) return launch_chunk(p);
  return MBS_OK;
}

mbs_status mbs_poll(mbs_plan p, int32_t slot, mbs_result* res) {
  if (!p || slot < 0 || slot >= p->nslots) return MBS_EINVAL;
  mbs_status st = progress(p, false);
  if (st != MBS_OK) return st;
  st = finish_poll(p, slot, res);
  if (st == MBS_EBUSY && res) {
    // progress of the running solve, as of the last completed launch
    const Slot& s = p->slots[slot];
    *res = mbs_result{};
    res->iterations = s.iter_seen;
    res->rel_residual = s.eps_seen;
    res->status = MBS_EBUSY;
  }
  return st;
}

mbs_status mbs_solve(mbs_plan p, int32_t slot, const void* src_dev, double tol, int32_t max_iter,
                     void* field_dev, mbs_result* res) {
  if (!field_dev) return MBS_EINVAL;
  mbs_status st = start_solve(p, slot, src_dev, tol, max_iter, field_dev);
  if (st != MBS_OK) return st;
  if (!p->in_flight) {
    st = launch_chunk(p);
    if (st != MBS_OK) return st;
  }
  for (;;) {
    st = progress(p, true);
    if (st != MBS_OK) return st;
    if (p->slots[slot].finishing) break;
  }
  HIP_TRY(hipEventSynchronize(p->slots[slot].done_ev));
  for (;;) {
    mbs_status r = finish_poll(p, slot, res);
    if (r != MBS_EBUSY) {
      HIP_TRY(hipStreamSynchronize(p->stream));
      return r;
    }
  }
}

mbs_status mbs_residual(mbs_plan p, int32_t slot, const void* field_dev, double* rel) {
  if (!p || slot < 0 || slot >= p->nslots || !rel) return MBS_EINVAL;
  Slot& s = p->slots[slot];
  if (!s.has_medium || !s.has_source || s.busy) return MBS_ESTATE;
  mbs_status st = push_desc(p, slot);
  if (st != MBS_OK) return st;
  double rho_ref = s.rho_ref;
  if (!(rho_ref > 0.0)) {
    if ((st = ensure_probe_x(p)) != MBS_OK) return st;
    HIP_TRY(launch_zero(p->probe_x, p->geo.vox, p->stream));
    if ((st = probe_norm(p, slot, p->probe_x, &rho_ref)) != MBS_OK) return st;
  }
  double rho = 0.0;
  if (field_dev) {
    if ((st = ensure_probe_x(p)) != MBS_OK) return st;
    HIP_TRY(launch_scatter((const float2*)field_dev, p->geo, p->probe_x, p->stream));
    st = probe_norm(p, slot, p->probe_x, &rho);
  } else {
    st = probe_norm(p, slot, s.x, &rho);
  }
  if (st != MBS_OK) return st;
  *rel = rho_ref > 0.0 ? rho / rho_ref : 0.0;
  return MBS_OK;
}

mbs_status mbs_residual_history(mbs_plan p, int32_t slot, double* out, int32_t max_n, int32_t* n) {
  if (!p || slot < 0 || slot >= p->nslots || !out || !n || max_n < 0) return MBS_EINVAL;
  const Slot& s = p->slots[slot];
  const int cnt = std::min(std::min(s.res.iterations, (int32_t)kHistCap), max_n);
  if (cnt > 0) {
    HIP_TRY(hipMemcpyAsync(out, s.hist, cnt * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  *n = cnt;
  return MBS_OK;
}

mbs_status mbs_timing_read(mbs_plan p, double* ms, int64_t* launches, int32_t n_kinds, int32_t reset) {
  if (!p || n_kinds < 0 || n_kinds > kKinds) return MBS_EINVAL;
  for (int k = 0; k < n_kinds; ++k) {
    if (ms) ms[k] = p->t_ms[k];
    if (launches) launches[k] = p->t_launch[k];
  }
  if (reset)
    for (int k = 0; k < kKinds; ++k) {
      p->t_ms[k] = 0;
      p->t_launch[k] = 0;
    }
  return MBS_OK;
}

}  // extern "C"
