// Internal structures shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbs {

constexpr int kThreads = 256;       // threads per workgroup of every kernel (4 wavefronts)
constexpr int kMaxT = 16;           // largest truncation t of the correction blocks
constexpr int kHistCap = 1 << 16;   // residual history entries kept per slot
constexpr int kReduceBlocks = 64;   // first-stage workgroups of the residual reduction
constexpr int kXferBlocks = 32;     // partial sums per subdomain of the transfer norms
constexpr int kMaxActSub = 4096;    // subdomains per plan when activation is on

// stop reasons written by the residual kernel
enum : int32_t {
  kRunning = 0,
  kConverged = 1,
  kMaxIter = 2,
  kDiverged = 3,
  kNonFinite = 4,
  kIdle = 5,        // slot not participating in the current launches
};

// Per-slot iteration state, read and written on the device.
struct SlotState {
  double rho_ref;   // ||Gamma^-1 y|| (set from iteration 0 when it is <= 0)
  double eps;       // relative residual of the last iteration
  double eps_prev;
  double rho;       // last residual norm
  double tol;
  int32_t iter;     // iterations completed
  int32_t max_iter;
  int32_t done;     // kRunning or a stop reason
  int32_t probe;    // 1: evaluate the residual once without updating the iterate
  double pad[2];
};

// Geometry of a plan (identical for every slot).
struct Geo {
  int32_t n[3];      // subdomain edge
  int32_t P[3];      // subdomains per axis
  int32_t a[3];      // a_d of Eq. 9 (0: no correction, 1: wrap removal, 2: split axis)
  int32_t periodic[3];
  int32_t N[3];      // global grid
  int32_t t;
  int32_t S;         // number of subdomains
  int64_t sub_vox;   // voxels per subdomain
  int64_t vox;       // voxels per slot (all subdomains)
  // face update: union of the edge slabs, split into disjoint regions per axis
  int64_t reg_count[3];  // voxels per subdomain in region d (0 if a_d == 0)
  int32_t reg_ext[3][3]; // extents of region d along each axis
  int32_t reg_off[3][3]; // offsets of region d along each axis (axis d itself: slab code)
  int64_t face_vox;      // sum of reg_count (per subdomain)
  int32_t cus;           // compute units of the device (persistent grid size)
  // layout of the work array W: z-line by z-line (wsh < 0), or in blocks of 2^wsh z values
  // (the slab schedule of the strided passes), element (s, i0, i1, j) at
  // s sub_vox + (j >> wsh) wplane + (i0 n1 + i1) 2^wsh + (j mod 2^wsh): one slab, one range
  int32_t wsh;
  int64_t wplane;        // n0 n1 2^wsh
};

// Per-slot pointers and scalars, in device memory (one table entry per slot).
struct SlotDesc {
  float2* x;              // iterate, subdomain-major [S][n0][n1][n2]
  float2* W;              // work array (FFTs in place; layout Geo::wsh)
  float2* W2;             // output of the inverse y pass in z-lines where W is blocked (Geo::wsh
                          // >= 0), read by the z pass; W itself otherwise
  float2* B;              // 1 - c (k^2 - k_b^2)
  float2* slab[3][4];     // per axis: 0 X (iterate edges), 1 U (edges of u), 2 Ex, 3 Eu
                          // each [S][2 sides][t][p][q]
  const float2* ybox;     // -c S on the source bounding box (global coordinates)
  int32_t ylo[3];
  int32_t yext[3];        // 0 extent: no source
  float c_im;             // c = i c_im
  float alpha;            // relaxation (0 in a probe evaluation)
  float kb2;
  float inv_vox;          // 1 / (n0 n1 n2)
  SlotState* st;
  double* part_main;      // residual partials of the last inverse pass
  double* part_face;      // residual partials of the face update
  double* hist;           // relative residual per iteration
  double* part_red;       // first-stage sums of the residual reduction (kReduceBlocks)
  const uint32_t* act;    // bit s set: subdomain s is iterated (nullptr: every subdomain)
  const int32_t* act_list;  // ids of the iterated subdomains, ascending (nullptr: all, in order)
  double* xfer;           // [S][kXferBlocks] partial sums of the field transferred into
                          // inactive subdomains (nullptr: activation off)
  int32_t n_act;          // entries of act_list
  // B of a lossless medium (Im n = 0 everywhere): only Im B is stored, one float per voxel, and
  // Re B = 1 + c_im k0^2 ramp(r) follows from the absorbing layers (bx_k = c_im k0^2; the ramp
  // of axis d rises by rstep[d] per voxel over the outer rw[d] voxels of each side)
  int32_t b_ramp;
  float bx_k;
  float rstep[3];
  int32_t rw[3];
};

// Part of a column pass: subdomains [sub0, sub0 + nsub) and z column chunks [cb0, cb0 + ncb) of
// the pass's tile width; ncb <= 0 means the whole pass over every subdomain.
struct ColRange {
  int32_t sub0, nsub, cb0, ncb;
};

// Launch helpers implemented in mbs_kernels.hip.
struct Tables {
  const float2* tw[3];    // forward twiddles exp(-2 pi i q / n_d), q < n_d
  const float* p2[3];     // |p_d|^2 per Fourier index (Nyquist at -pi)
  const float* C;         // t x t correction block (row-major C[a][b])
};

int lines_per_wg(int n);   // contiguous passes: lines per workgroup
bool fft_size_supported(int n);

hipError_t launch_first_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                             hipStream_t s);
void prepare_launches(const Geo& g);
hipError_t launch_xfer(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, hipStream_t s);
hipError_t launch_mid_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                           int inverse, hipStream_t s, ColRange rg = ColRange{0, 0, 0, 0});
hipError_t launch_green_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                             hipStream_t s, ColRange rg = ColRange{0, 0, 0, 0});
int col_chunk_width(int n, int kind);  // z columns per tile of a column pass
hipError_t launch_last_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                            hipStream_t s);
hipError_t launch_corr(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, int which,
                       hipStream_t s, int axis_mask = 7);
// fused z passes (see mbs_kernels.hip)
bool fusion_supported(const Geo& g);
int host_slab_line_count(const Geo& g);
int64_t slabA_blocks(const Geo& g);
hipError_t launch_fused(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, hipStream_t s);
hipError_t launch_wpass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, int slab_only,
                        hipStream_t s);
hipError_t launch_slabA(const SlotDesc* tab, int nslots, const Geo& g, hipStream_t s);
hipError_t launch_face(const SlotDesc* tab, int nslots, const Geo& g, hipStream_t s);
hipError_t launch_reduce(const SlotDesc* tab, int nslots, const Geo& g, int64_t n_main,
                         int64_t n_face, hipStream_t s);
int64_t last_pass_blocks(const Geo& g);
int64_t face_blocks(const Geo& g);

// set-up kernels
struct MediumStats {
  double re_min, re_max, im_min;
  double nonfinite;
  double nim_max;  // max |Im n| (0: a lossless medium)
};
hipError_t launch_medium_stats(const float2* n, const Geo& g, double k0sq, const int32_t* width,
                               double ramp_max, MediumStats* partials, int64_t nblocks,
                               hipStream_t s);
hipError_t launch_medium_kmax(const float2* n, const Geo& g, double k0sq, const int32_t* width,
                              double ramp_max, double kb2, double* partials, int64_t nblocks,
                              hipStream_t s);
hipError_t launch_medium_B(const float2* n, const Geo& g, double k0sq, const int32_t* width,
                           double ramp_max, double kb2, double c_im, float2* B, int compact, hipStream_t s);
int64_t setup_blocks(const Geo& g);
hipError_t launch_source_bbox(const float2* S, const Geo& g, int32_t* bbox /*lo3,hi3,nonfinite*/,
                              hipStream_t s);
hipError_t launch_source_fill(const float2* S, const Geo& g, const int32_t* lo, const int32_t* ext,
                              double c_im, float2* ybox, hipStream_t s);
hipError_t launch_scatter(const float2* field, const Geo& g, float2* x, hipStream_t s);
hipError_t launch_gather(const float2* x, const Geo& g, float2* field, hipStream_t s);
hipError_t launch_zero(float2* p, int64_t n, hipStream_t s);
hipError_t put_state(SlotState* dst, const SlotState& v, hipStream_t s);
hipError_t put_desc(SlotDesc* dst, const SlotDesc& v, hipStream_t s);
hipError_t put_i32x8(int32_t* dst, const int32_t* v, hipStream_t s);
hipError_t launch_extract_slabs(const SlotDesc* tab, int slot, const Geo& g, int which,
                                hipStream_t s);

}  // namespace mbs
