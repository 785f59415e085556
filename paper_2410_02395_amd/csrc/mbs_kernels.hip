// HIP kernels (gfx950) of the modified Born series iteration with domain
// decomposition (Mache & Vellekoop, arXiv 2410.02395).
//
// One iteration of Eq. 6 on every subdomain of every active slot (default sequence):
//   k_col<.,0>  FFT along y of w                           (Eq. 5)
//   k_col<.,2>  FFT along x, multiply by the (L+I)^-1 symbol, inverse FFT along x
//   k_col<.,1>  inverse FFT along y (into W2, in z-lines, where W is stored slab by slab)
//               (the three column passes run whole, or subdomain by subdomain on z slabs
//               that stay in the memory-side cache between them)
//   k_fused     per global z-line: inverse FFT along z, u = x - v, d = B u + z-edge terms,
//               x -= alpha d, FP64 residual partials; then w of the next iteration,
//               y + B x + z-edge terms, and its forward FFT along z  (Eq. 6, Sec. 3.1)
//   k_corr      x/y edge corrections of u; k_slabA finishes the x/y edge-slab lines
//   k_corr      x/y edge corrections of the new x; k_wpass forms w on the edge-slab lines
//   reduce      rho_n = ||d_n|| in FP64, eps_n, stop test  (Sec. 3.1 stop rule)
// A separate sequence (k_first, k_last, k_face: first forward and last inverse z pass
// apart) serves plans that do not fuse and the residual evaluation.  The FFTs are
// Stockham autosort passes (radix 8/4/3/2) over tiles staged in LDS: whole lines along
// the contiguous axis, or N x WC column tiles along a strided axis, so every global
// access is a coalesced row of >= 64 bytes.  No MFMA: nothing here is a dense
// contraction; the path is HBM-bound.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mbs_internal.h"

namespace mbs {

// Pointers read from the slot table are generic; casting them to the global address
// space makes the compiler emit global (not flat) loads and stores, which do not
// count against the LDS wait counter and so stay in flight across LDS barriers.
// Small tables that no kernel writes while it runs (the list of iterated subdomains) are read
// through the constant address space instead: uniform reads then become scalar loads, which
// do not count against the vector-memory wait counter of the streaming loops.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cp(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}
#else
template <class T>
__device__ __forceinline__ T* gp(T* p) {  // host pass: parsed only, never executed
  return p;
}
template <class T>
__device__ __forceinline__ const T* cp(const T* p) {
  return p;
}
#endif

// Streaming loads and stores: with NT they carry the nontemporal hint (data that the kernel
// touches once and that no later kernel of the iteration finds in a cache).
#if defined(__HIP_DEVICE_COMPILE__)
typedef float f2v __attribute__((ext_vector_type(2)));
template <bool NT, class P>
__device__ __forceinline__ float2 ld_g(P p) {
  if constexpr (NT) {
    const f2v v = __builtin_nontemporal_load((const __attribute__((address_space(1))) f2v*)p);
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT, class P>
__device__ __forceinline__ void st_g(P p, float2 v) {
  if constexpr (NT) {
    const f2v w = {v.x, v.y};
    __builtin_nontemporal_store(w, (__attribute__((address_space(1))) f2v*)p);
  } else {
    *p = v;
  }
}
template <bool NT, class P>
__device__ __forceinline__ float ld_gf(P p) {
  if constexpr (NT) return __builtin_nontemporal_load((const __attribute__((address_space(1))) float*)p);
  else return *p;
}
#else
template <bool NT, class P>
__device__ __forceinline__ float ld_gf(P p) { return *p; }
template <bool NT, class P>
__device__ __forceinline__ float2 ld_g(P p) { return *p; }
template <bool NT, class P>
__device__ __forceinline__ void st_g(P p, float2 v) { *p = v; }
#endif
// The z-line passes read and write each element once per iteration: their loads and stores
// take the nontemporal hint (about 3 % faster on the fused z pass; MBS_LINE_NT=0 drops it).
#ifndef MBS_LINE_NT
#define MBS_LINE_NT 1
#endif
template <class P>
__device__ __forceinline__ float2 ld_line(P p) { return ld_g<MBS_LINE_NT != 0>(p); }
template <class P>
__device__ __forceinline__ void st_line(P p, float2 v) { st_g<MBS_LINE_NT != 0>(p, v); }
// The column passes: the x pass reads what the forward y pass wrote, and the inverse y pass what
// the x pass wrote, from the memory-side cache when they run slab by slab, so those loads and
// stores stay cached.  The inverse y pass's stores are read back only by the next z pass, after
// the whole array has streamed: at 512-point columns they take the nontemporal hint (about 2 %
// faster there; at 256 points the hint costs about 1 %).
__host__ __device__ constexpr bool col_ld_nt(int) { return false; }
__host__ __device__ constexpr bool col_st_nt(int kind, int n) { return kind == 1 && n >= 512; }

// ---------------------------------------------------------------------------
// complex helpers (float2 = interleaved re, im)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  // explicit fma order: the same product rounds the same way in every kernel
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// |a|^2 in FP64 (the residual sums)
__device__ __forceinline__ double norm2d(float2 a) { return fma((double)a.x, (double)a.x, (double)a.y * a.y); }
// multiply by i*SIGN  (SIGN = -1: -i, SIGN = +1: +i)
template <int SIGN>
__device__ __forceinline__ float2 mul_si(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// (-c) z with c = i c_im
__device__ __forceinline__ float2 mul_negc(float2 z, float c_im) {
  return make_float2(c_im * z.y, -c_im * z.x);
}

// ---------------------------------------------------------------------------
// DFT butterflies; SIGN = -1 forward (exp(-2 pi i jk/R)), +1 inverse
// ---------------------------------------------------------------------------
template <int SIGN, int R>
struct Bfly;

template <int SIGN>
struct Bfly<SIGN, 2> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
};

template <int SIGN>
struct Bfly<SIGN, 3> {
  __device__ __forceinline__ static void run(float2* v) {
    const float h = 0.86602540378443864676f;  // sqrt(3)/2
    float2 s = cadd(v[1], v[2]);
    float2 d = mul_si<SIGN>(csub(v[1], v[2]));
    float2 t = make_float2(fmaf(-0.5f, s.x, v[0].x), fmaf(-0.5f, s.y, v[0].y));
    v[0] = cadd(v[0], s);
    v[1] = make_float2(fmaf(h, d.x, t.x), fmaf(h, d.y, t.y));
    v[2] = make_float2(fmaf(-h, d.x, t.x), fmaf(-h, d.y, t.y));
  }
};

template <int SIGN>
struct Bfly<SIGN, 4> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]);
    float2 t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]);
    float2 t3 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

// radix 8 as two radix-4 butterflies: the even outputs from a_m = v_m + v_{m+4}, the odd
// ones from b_m = (v_m - v_{m+4}) w8^(SIGN m), w8 = exp(i pi/4).  w8^S b_1 and w8^3S b_3 enter
// the odd radix-4 butterfly only as their sum and difference, each one rounding of an fma.
template <int SIGN>
struct Bfly<SIGN, 8> {
  __device__ __forceinline__ static void run(float2* v) {
    const float r = 0.70710678118654752440f;
    float2 a[4], b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      a[m] = cadd(v[m], v[m + 4]);
      b[m] = csub(v[m], v[m + 4]);
    }
    Bfly<SIGN, 4>::run(a);
    const float2 z1 = b[1], z3 = b[3];
    // w8^S z1 = r u1, w8^3S z3 = r u3
    const float2 u1 = SIGN > 0 ? make_float2(z1.x - z1.y, z1.x + z1.y) : make_float2(z1.x + z1.y, z1.y - z1.x);
    const float2 u3 = SIGN > 0 ? make_float2(-(z3.x + z3.y), z3.x - z3.y) : make_float2(z3.y - z3.x, -(z3.x + z3.y));
    const float2 p1 = make_float2(r * u1.x, r * u1.y);
    const float2 s13 = make_float2(fmaf(r, u3.x, p1.x), fmaf(r, u3.y, p1.y));
    const float2 d13 = mul_si<SIGN>(make_float2(fmaf(-r, u3.x, p1.x), fmaf(-r, u3.y, p1.y)));
    const float2 b2 = mul_si<SIGN>(b[2]);
    const float2 t0 = cadd(b[0], b2), t1 = csub(b[0], b2);
    v[0] = a[0]; v[2] = a[1]; v[4] = a[2]; v[6] = a[3];
    v[1] = cadd(t0, s13);
    v[5] = csub(t0, s13);
    v[3] = cadd(t1, d13);
    v[7] = csub(t1, d13);
  }
};

// radix of the next Stockham stage for the remaining length
__host__ __device__ constexpr int radix_of(int rem) {
  return rem % 3 == 0 ? 3 : (rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : 2));
}
__host__ __device__ constexpr int plan_len(int n) {
  int c = 0;
  while (n > 1) {
    n /= radix_of(n);
    ++c;
  }
  return c;
}
__host__ __device__ constexpr int radix_at(int n, int s) {
  for (int k = 0; k < s; ++k) n /= radix_of(n);
  return radix_of(n);
}
// radix of stage s of the forward (rev = false) or reversed (rev = true) radix sequence
__host__ __device__ constexpr int plan_radix(int n, int s, bool rev) {
  return radix_at(n, rev ? plan_len(n) - 1 - s : s);
}
// product of the radices before stage s (the length of the sub-transforms already done)
__host__ __device__ constexpr int plan_ns(int n, int s, bool rev) {
  int p = 1;
  for (int k = 0; k < s; ++k) p *= plan_radix(n, k, rev);
  return p;
}

// keeps registers allocated up to this point (no instruction is emitted); used so that the
// next tile's loads do not land in registers a pending store still has to read
template <int PER, int R>
__device__ __forceinline__ void keep_alive(const float2 (&v)[PER][R]) {
#pragma unroll
  for (int q = 0; q < PER; ++q)
#pragma unroll
    for (int m = 0; m < R; ++m) asm volatile("" ::"v"(v[q][m].x), "v"(v[q][m].y));
}

// barrier for LDS traffic only: waits for this wave's LDS operations, not for its
// outstanding global loads, so prefetches stay in flight across FFT stages
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ---------------------------------------------------------------------------
// tile layouts in LDS
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int lines_per_wg_c(int n) { return n >= 2048 ? 1 : 2048 / n; }
__host__ __device__ constexpr int cols_per_tile_c(int n) {
  return n >= 768 ? 8 : (n >= 128 ? 16 : (n >= 64 ? 32 : 64));
}

// LINES whole lines of N contiguous elements; element (j, l) at l*N + j, padded by one
// slot every 2^MBS_LINE_PAD to spread the strided writes of the Stockham stages over the banks.
#ifndef MBS_LINE_PAD
#define MBS_LINE_PAD 4
#endif
template <int N, int LINES>
struct LineTile {
  static constexpr int NT = kThreads;
  static constexpr int ELEMS = N * LINES;
  static constexpr int LDS = ELEMS + (ELEMS >> MBS_LINE_PAD) + 1;
  __device__ __forceinline__ static int idx(int j, int l) {
    int f = l * N + j;
    return f + (f >> MBS_LINE_PAD);
  }
  template <int R>
  __device__ __forceinline__ static void bf(int b, int& i, int& l) {
    i = b % (N / R);
    l = b / (N / R);
  }
  template <int R>
  static constexpr int nb() { return (N / R) * LINES; }
};

// threads of the y-pass column tiles for 384 <= n <= 512: 1024 (8 elements per thread, 87 VGPRs,
// 16 waves per CU) against 512 (16 elements, 162 VGPRs, 8 waves): 3.7 % faster strided passes
#ifndef MBS_COLY_NT
#define MBS_COLY_NT 1024
#endif
// threads of the column tiles for n >= 768 (8 columns): 1024 (8 elements per thread, 81-120 VGPRs)
// against 512 (16 elements, 163-214 VGPRs): 6.6 % faster strided passes on 1024-point axes
#ifndef MBS_COLBIG_NT
#define MBS_COLBIG_NT 1024
#endif
__host__ __device__ constexpr int col_threads_c(int n) {
  return n >= 768 ? MBS_COLBIG_NT : (n >= 384 ? MBS_COLY_NT : kThreads);
}
// minimum waves per SIMD requested for the column tiles (register budget per thread)
#ifndef MBS_COL_WAVES_BIG
#define MBS_COL_WAVES_BIG 2
#endif
__host__ __device__ constexpr int col_waves_c(int n) {
  return col_threads_c(n) == 1024 ? 4 : (col_threads_c(n) == 512 ? MBS_COL_WAVES_BIG : 2);
}
// 1: the next tile's loads are issued before the current tile's FFT stages
#ifndef MBS_COL_PREFETCH
#define MBS_COL_PREFETCH 1
#endif
// parts in which the next tile's loads are issued over an iteration of the persistent column
// loop: x pass (two FFTs) and y passes (one FFT)
#ifndef MBS_GREEN_SPLIT
#define MBS_GREEN_SPLIT 3
#endif
#ifndef MBS_COL_SPLIT
#define MBS_COL_SPLIT 1
#endif
// tile shape of the x pass (two FFTs per column) for MBS_GREEN_MIN_N <= N <= 512 (half the
// threads below 384: eight elements per thread either way)
#ifndef MBS_GREEN_WC
#define MBS_GREEN_WC 16
#endif
#ifndef MBS_GREEN_NT
#define MBS_GREEN_NT 1024
#endif
#ifndef MBS_GREEN_WAVES
#define MBS_GREEN_WAVES 4
#endif
#ifndef MBS_GREEN_MIN_N
#define MBS_GREEN_MIN_N 256
#endif
__host__ __device__ constexpr bool green_tile_c(int n, int kind) {
  return kind == 2 && n >= MBS_GREEN_MIN_N && n <= 512;
}
// per pass kind: columns per tile, threads per workgroup, minimum waves per SIMD
__host__ __device__ constexpr int col_wc_c(int n, int kind) {
  return green_tile_c(n, kind) ? MBS_GREEN_WC : cols_per_tile_c(n);
}
__host__ __device__ constexpr int col_nt_c(int n, int kind) {
  return green_tile_c(n, kind) ? (n < 384 ? MBS_GREEN_NT / 2 : MBS_GREEN_NT) : col_threads_c(n);
}
__host__ __device__ constexpr int col_wv_c(int n, int kind) {
  return green_tile_c(n, kind) ? MBS_GREEN_WAVES : col_waves_c(n);
}

// N rows (the FFT axis) x WC contiguous columns, NTH threads; element (j, c) at j*WC + c.
template <int N, int WC, int NTH>
struct ColTile {
  static constexpr int NT = NTH;
  static constexpr int ELEMS = N * WC;
  static constexpr int LDS = ELEMS;
  __device__ __forceinline__ static int idx(int j, int c) { return j * WC + c; }
  template <int R>
  __device__ __forceinline__ static void bf(int b, int& i, int& c) {
    c = b % WC;
    i = b / WC;
  }
  template <int R>
  static constexpr int nb() { return (N / R) * WC; }
};

// butterflies per thread in a stage of radix R
template <class Tile, int R>
__host__ __device__ constexpr int per_thread() { return (Tile::template nb<R>() + Tile::NT - 1) / Tile::NT; }

template <class Tile, int R>
__device__ __forceinline__ bool bvalid(int q, int tid) {
  constexpr int NB = Tile::template nb<R>();
  return (NB % Tile::NT) == 0 || tid + q * Tile::NT < NB;
}

// Stockham stage (radix R, NS = length of the sub-transforms already done): butterfly i
// (of N/R per line) takes elements i + m N/R, multiplies input m by w^(m k) with
// k = i mod NS and w = exp(SIGN 2 pi i / (NS R)), and produces outputs at
// (i - k) R + k + m NS.  The data of butterfly q of this thread is v[q][0..R).
template <class Tile, int N, int R, int NS, int SIGN, int PER>
__device__ __forceinline__ void bfly_regs(float2 (&v)[PER][R], const float2* __restrict__ tw, int tid) {
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (!bvalid<Tile, R>(q, tid)) continue;
    if constexpr (NS > 1) {
      int i, l;
      Tile::template bf<R>(tid + q * Tile::NT, i, l);
      const int k = i % NS;
#pragma unroll
      for (int m = 1; m < R; ++m) {
        float2 w = tw[(m * k) * (N / (NS * R))];
        if (SIGN > 0) w.y = -w.y;
        v[q][m] = cmul(v[q][m], w);
      }
    }
    Bfly<SIGN, R>::run(v[q]);
  }
}

template <class Tile, int N, int R, int NS, int PER>
__device__ __forceinline__ void put_lds(float2* lds, const float2 (&v)[PER][R], int tid) {
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (!bvalid<Tile, R>(q, tid)) continue;
    int i, l;
    Tile::template bf<R>(tid + q * Tile::NT, i, l);
    const int k = i % NS;
    const int o = (i - k) * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) lds[Tile::idx(o + m * NS, l)] = v[q][m];
  }
}

template <class Tile, int N, int R, int PER>
__device__ __forceinline__ void get_lds(const float2* lds, float2 (&v)[PER][R], int tid) {
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (!bvalid<Tile, R>(q, tid)) continue;
    int i, l;
    Tile::template bf<R>(tid + q * Tile::NT, i, l);
#pragma unroll
    for (int m = 0; m < R; ++m) v[q][m] = lds[Tile::idx(i + m * (N / R), l)];
  }
}

// stages S .. SEND-1 of the plan, in place in LDS
template <class Tile, int N, bool REV, int SIGN, int S, int SEND>
__device__ __forceinline__ void lds_stages(float2* lds, const float2* __restrict__ tw, int tid) {
  if constexpr (S < SEND) {
    constexpr int R = plan_radix(N, S, REV);
    constexpr int NS = plan_ns(N, S, REV);
    constexpr int PER = per_thread<Tile, R>();
    float2 v[PER][R];
    get_lds<Tile, N, R, PER>(lds, v, tid);
    bfly_regs<Tile, N, R, NS, SIGN, PER>(v, tw, tid);
    lds_barrier();
    put_lds<Tile, N, R, NS, PER>(lds, v, tid);
    lds_barrier();
    lds_stages<Tile, N, REV, SIGN, S + 1, SEND>(lds, tw, tid);
  }
}

// First stage of an FFT: butterflies of `in` (stage-0 inputs, elements i + m N/R0 of this
// thread's butterflies) in registers, outputs written to LDS.  Starts with a barrier so the
// caller may have been reading LDS just before.  For a one-stage plan nothing goes to LDS.
template <class Tile, int N, bool REV, int SIGN, int PER0, int R0>
__device__ __forceinline__ void fft_head(float2 (&in)[PER0][R0], float2* lds, const float2* __restrict__ tw,
                                         int tid) {
  constexpr int P = plan_len(N);
  static_assert(R0 == plan_radix(N, 0, REV), "plan mismatch");
  bfly_regs<Tile, N, R0, 1, SIGN, PER0>(in, tw, tid);
  if constexpr (P > 1) {
    lds_barrier();
    put_lds<Tile, N, R0, 1, PER0>(lds, in, tid);
    lds_barrier();
  }
}

// Remaining stages: the middle ones in LDS, the last one read into `out` (outputs at
// i + m N/RL, natural order).  For a one-stage plan `in` already holds the result.
template <class Tile, int N, bool REV, int SIGN, int PER0, int R0, int PERL, int RL>
__device__ __forceinline__ void fft_tail(float2 (&in)[PER0][R0], float2 (&out)[PERL][RL], float2* lds,
                                         const float2* __restrict__ tw, int tid) {
  constexpr int P = plan_len(N);
  static_assert(RL == plan_radix(N, P - 1, REV), "plan mismatch");
  if constexpr (P == 1) {
#pragma unroll
    for (int q = 0; q < PER0; ++q)
#pragma unroll
      for (int m = 0; m < R0; ++m) out[q][m] = in[q][m];
  } else {
    lds_stages<Tile, N, REV, SIGN, 1, P - 1>(lds, tw, tid);
    get_lds<Tile, N, RL, PERL>(lds, out, tid);
    bfly_regs<Tile, N, RL, plan_ns(N, P - 1, REV), SIGN, PERL>(out, tw, tid);
  }
}

// Whole FFT of a tile (head then tail).
template <class Tile, int N, bool REV, int SIGN, int PER0, int R0, int PERL, int RL>
__device__ __forceinline__ void fft_tile(float2 (&in)[PER0][R0], float2 (&out)[PERL][RL], float2* lds,
                                         const float2* __restrict__ tw, int tid) {
  fft_head<Tile, N, REV, SIGN, PER0, R0>(in, lds, tw, tid);
  fft_tail<Tile, N, REV, SIGN, PER0, R0, PERL, RL>(in, out, lds, tw, tid);
}

// ---------------------------------------------------------------------------
// block reduction of one double per thread (fixed order: deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  }
  return s;  // valid on thread 0
}

// ---------------------------------------------------------------------------
// per-line bookkeeping of the contiguous (z) passes
// ---------------------------------------------------------------------------
struct LineInfo {
  int64_t gbase;   // index of element 0 of the line in the subdomain-major arrays
  int64_t wbase;   // the same in the layout of W (w_off)
  int64_t e0;      // slab offset for axis 0 (element j at e0 + j), -1 if not in a slab
  int64_t e1;      // slab offset for axis 1, -1 if not in a slab
  int64_t e2;      // slab offset for axis 2 at depth 0 of side 0 (-1: axis not corrected)
  int64_t ybase;   // source box index of element j (ybase + j), valid for j in [jlo, jhi)
  int32_t jlo, jhi;
  int32_t valid;
  int32_t on;      // the line's subdomain is iterated (subdomain activation, Sec. 3.1)
  float r01;       // absorbing ramp of the line's x and y position (compact B)
  int32_t gz0;     // global z of element 0
};

// W index of element 0 of the z-line (i0, i1) of subdomain s
__device__ __forceinline__ int64_t w_line_base(int s, int i0, int i1, const Geo& g) {
  const int64_t k = (int64_t)i0 * g.n[1] + i1;
  return (int64_t)s * g.sub_vox + (g.wsh < 0 ? k * g.n[2] : k << g.wsh);
}
// offset of z index j from element 0 of its line (within one subdomain: below 2^31)
__device__ __forceinline__ int32_t w_off(int j, const Geo& g) {
  return g.wsh < 0 ? j : (j >> g.wsh) * (int32_t)g.wplane + (j & ((1 << g.wsh) - 1));
}
__device__ __forceinline__ int64_t w_at(int64_t wbase, int j, const Geo& g) { return wbase + w_off(j, g); }
// Elements i + m S of a line with i < S (S = N/R: a thread's elements in a radix-R stage): W is
// blocked only when n_2 and the block height are powers of two, so one of S and the block
// height divides the other and w_off(i + m S) = w_off(i) + w_off(m S), a per-lane part and a
// part that is the same for every lane.

// Absorbing ramp of global index i along axis d, as the medium set-up applies it (Sec. 4: the
// outer rw[d] voxels of each side, rising linearly to the boundary)
__device__ __forceinline__ float ramp_axis(const SlotDesc& sd, const Geo& g, int d, int i) {
  const int W = sd.rw[d];
  float r = 0.f;
  if (i < W) r = sd.rstep[d] * (float)(W - i);
  if (i >= g.N[d] - W) r = fmaxf(r, sd.rstep[d] * (float)(i - (g.N[d] - W) + 1));
  return r;
}

// B = 1 - c (k^2 - k_b^2) at element j (index gi) of a line: stored whole, or for a lossless
// medium Im B stored and Re B = 1 + c_im k0^2 ramp(r) from the line's position
__device__ __forceinline__ float2 b_line(const SlotDesc& sd, const Geo& g, const LineInfo& li, int j, int64_t gi) {
  if (sd.b_ramp) {
    const float r = fmaxf(li.r01, ramp_axis(sd, g, 2, li.gz0 + j));
    return make_float2(fmaf(sd.bx_k, r, 1.f), gp(reinterpret_cast<const float*>(sd.B))[gi]);
  }
  return gp(sd.B)[gi];
}

// subdomain s is iterated (all are when no activation mask is set)
__device__ __forceinline__ bool sub_on(const uint32_t* act, int s) {
  return act == nullptr || ((act[s >> 5] >> (s & 31)) & 1u) != 0u;
}

__device__ __forceinline__ void line_info(int64_t line, const Geo& g, const SlotDesc& sd,
                                          LineInfo& li) {
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2], t = g.t;
  const int64_t nlines = (int64_t)g.S * n0 * n1;
  li.valid = line < nlines;
  li.on = 0;
  li.r01 = 0.f;
  li.gz0 = 0;
  if (!li.valid) return;
  int i0, i1, s;
  if (nlines <= (int64_t)UINT32_MAX) {
    // 32-bit division where the line index fits: a fraction of the 64-bit sequence
    const uint32_t u = (uint32_t)line, r = u / (uint32_t)n1;
    i1 = (int)(u - r * (uint32_t)n1);
    s = (int)(r / (uint32_t)n0);
    i0 = (int)(r - (uint32_t)s * (uint32_t)n0);
  } else {
    const int64_t r = line / n1;
    i1 = (int)(line - r * n1);
    s = (int)(r / n0);
    i0 = (int)(r - (int64_t)s * n0);
  }
  {
    const int c2 = s % g.P[2], c1 = (s / g.P[2]) % g.P[1], c0 = s / (g.P[2] * g.P[1]);
    li.r01 = fmaxf(ramp_axis(sd, g, 0, c0 * n0 + i0), ramp_axis(sd, g, 1, c1 * n1 + i1));
    li.gz0 = c2 * n2;
  }
  li.on = sub_on(sd.act, s) ? 1 : 0;
  li.gbase = line * n2;
  li.wbase = w_line_base(s, i0, i1, g);
  li.e0 = -1;
  li.e1 = -1;
  li.e2 = -1;
  if (g.a[0] > 0 && (i0 < t || i0 >= n0 - t)) {
    const int side = i0 < t ? 0 : 1;
    const int aa = side ? i0 - (n0 - t) : i0;
    li.e0 = (((int64_t)s * 2 + side) * t + aa) * ((int64_t)n1 * n2) + (int64_t)i1 * n2;
  }
  if (g.a[1] > 0 && (i1 < t || i1 >= n1 - t)) {
    const int side = i1 < t ? 0 : 1;
    const int aa = side ? i1 - (n1 - t) : i1;
    li.e1 = (((int64_t)s * 2 + side) * t + aa) * ((int64_t)n0 * n2) + (int64_t)i0 * n2;
  }
  if (g.a[2] > 0) li.e2 = ((int64_t)s * 2 * t) * ((int64_t)n0 * n1) + (int64_t)i0 * n1 + i1;
  // source box (global coordinates)
  li.jlo = 0;
  li.jhi = 0;
  li.ybase = 0;
  if (sd.yext[0] > 0) {
    const int s2 = s % g.P[2];
    const int s1 = (s / g.P[2]) % g.P[1];
    const int s0 = s / (g.P[2] * g.P[1]);
    const int g0 = s0 * n0 + i0 - sd.ylo[0];
    const int g1 = s1 * n1 + i1 - sd.ylo[1];
    if (g0 >= 0 && g0 < sd.yext[0] && g1 >= 0 && g1 < sd.yext[1]) {
      const int z0 = s2 * n2;  // global z of local j = 0
      int lo = sd.ylo[2] - z0;
      int hi = sd.ylo[2] + sd.yext[2] - z0;
      lo = lo < 0 ? 0 : lo;
      hi = hi > n2 ? n2 : hi;
      if (lo < hi) {
        li.jlo = lo;
        li.jhi = hi;
        li.ybase = ((int64_t)g0 * sd.yext[1] + g1) * sd.yext[2] + (z0 - sd.ylo[2]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// first pass: w = y + B x + sum_d Ex_d, forward FFT along z
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kThreads) void k_first(const SlotDesc* __restrict__ tab, Geo g,
                                                    Tables tb) {
  const SlotDesc sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  constexpr int L = lines_per_wg_c(N);
  using Tile = LineTile<N, L>;
  constexpr int P = plan_len(N);
  constexpr int R0 = plan_radix(N, 0, false), RL = plan_radix(N, P - 1, false);
  constexpr int PER0 = per_thread<Tile, R0>(), PERL = per_thread<Tile, RL>();
  __shared__ float2 lds[Tile::LDS];
  __shared__ LineInfo info[L];
  const int tid = threadIdx.x;
  const int64_t line0 = (int64_t)blockIdx.x * L;
  for (int l = tid; l < L; l += kThreads) line_info(line0 + l, g, sd, info[l]);
  __syncthreads();
  const int t = g.t;
  const int64_t plane2 = (int64_t)g.n[0] * g.n[1];
  const auto X = gp(sd.x);
  const auto E0 = gp(sd.slab[0][2]);
  const auto E1 = gp(sd.slab[1][2]);
  const auto E2 = gp(sd.slab[2][2]);
  const auto Y = gp(sd.ybox);
  const auto W = gp(sd.W);
  float2 v[PER0][R0];
#pragma unroll
  for (int q = 0; q < PER0; ++q) {
    int i = 0, l = 0;
    const bool ok = bvalid<Tile, R0>(q, tid);
    if (ok) Tile::template bf<R0>(tid + q * kThreads, i, l);
    const LineInfo& li = info[ok ? l : 0];
#pragma unroll
    for (int m = 0; m < R0; ++m) {
      const int j = i + m * (N / R0);
      float2 w = make_float2(0.f, 0.f);
      if (ok && li.valid) {
        const int64_t gi = li.gbase + j;
        w = cmul(b_line(sd, g, li, j, gi), X[gi]);
        if (li.e0 >= 0) w = cadd(w, E0[li.e0 + j]);
        if (li.e1 >= 0) w = cadd(w, E1[li.e1 + j]);
        if (li.e2 >= 0) {
          if (j < t) w = cadd(w, E2[li.e2 + (int64_t)j * plane2]);
          else if (j >= N - t) w = cadd(w, E2[li.e2 + (int64_t)(t + j - (N - t)) * plane2]);
        }
        if (j >= li.jlo && j < li.jhi) w = cadd(w, Y[li.ybase + j]);
      }
      v[q][m] = w;
    }
  }
  float2 o[PERL][RL];
  fft_tile<Tile, N, false, -1>(v, o, lds, tb.tw[2], tid);
#pragma unroll
  for (int q = 0; q < PERL; ++q) {
    if (!bvalid<Tile, RL>(q, tid)) continue;
    int i, l;
    Tile::template bf<RL>(tid + q * kThreads, i, l);
    if (!info[l].valid) continue;
    const auto p = W + (info[l].wbase + w_off(i, g));
#pragma unroll
    for (int m = 0; m < RL; ++m) st_line(p + w_off(m * (N / RL), g), o[q][m]);
  }
}

// ---------------------------------------------------------------------------
// last pass: inverse FFT along z, u = x - v, x -= alpha B u, edge slabs of u,
// residual partial sum of |B u|^2 over voxels outside every edge slab
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kThreads) void k_last(const SlotDesc* __restrict__ tab, Geo g,
                                                   Tables tb) {
  const SlotDesc sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  constexpr int L = lines_per_wg_c(N);
  using Tile = LineTile<N, L>;
  constexpr int P = plan_len(N);
  constexpr int R0 = plan_radix(N, 0, false), RL = plan_radix(N, P - 1, false);
  constexpr int PER0 = per_thread<Tile, R0>(), PERL = per_thread<Tile, RL>();
  __shared__ float2 lds[Tile::LDS];
  __shared__ LineInfo info[L];
  __shared__ double red[kThreads / 64];
  const int tid = threadIdx.x;
  const int64_t line0 = (int64_t)blockIdx.x * L;
  for (int l = tid; l < L; l += kThreads) line_info(line0 + l, g, sd, info[l]);
  __syncthreads();
  const auto X = gp(sd.x);
  const auto W2 = gp(sd.W2);  // output of the inverse y pass, in z-lines
  const auto U0 = gp(sd.slab[0][1]);
  const auto U1 = gp(sd.slab[1][1]);
  const auto U2 = gp(sd.slab[2][1]);
  float2 v[PER0][R0];
#pragma unroll
  for (int q = 0; q < PER0; ++q) {
    int i = 0, l = 0;
    const bool ok = bvalid<Tile, R0>(q, tid);
    if (ok) Tile::template bf<R0>(tid + q * kThreads, i, l);
    const LineInfo& li = info[ok ? l : 0];
#pragma unroll
    for (int m = 0; m < R0; ++m)
      v[q][m] = (ok && li.valid) ? W2[li.gbase + i + m * (N / R0)] : make_float2(0.f, 0.f);
  }
  float2 o[PERL][RL];
  fft_tile<Tile, N, false, +1>(v, o, lds, tb.tw[2], tid);
  const int t = g.t;
  const int64_t plane2 = (int64_t)g.n[0] * g.n[1];
  const float alpha = sd.alpha;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < PERL; ++q) {
    if (!bvalid<Tile, RL>(q, tid)) continue;
    int i, l;
    Tile::template bf<RL>(tid + q * kThreads, i, l);
    const LineInfo& li = info[l];
    if (!li.valid) continue;
#pragma unroll
    for (int m = 0; m < RL; ++m) {
      const int j = i + m * (N / RL);
      const int64_t gi = li.gbase + j;
      const float2 xv = X[gi];
      const float2 u = csub(xv, o[q][m]);
      const float2 bu = cmul(b_line(sd, g, li, j, gi), u);
      X[gi] = make_float2(fmaf(-alpha, bu.x, xv.x), fmaf(-alpha, bu.y, xv.y));
      bool edge = false;
      if (li.e0 >= 0) { U0[li.e0 + j] = u; edge = true; }
      if (li.e1 >= 0) { U1[li.e1 + j] = u; edge = true; }
      if (li.e2 >= 0) {
        if (j < t) { U2[li.e2 + (int64_t)j * plane2] = u; edge = true; }
        else if (j >= N - t) { U2[li.e2 + (int64_t)(t + j - (N - t)) * plane2] = u; edge = true; }
      }
      if (!edge) acc += norm2d(bu);
    }
  }
  const double s = block_sum(acc, red);
  if (tid == 0) gp(sd.part_main)[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// strided passes over N x WC column tiles: FFT along y (KIND 0 forward, 1 inverse)
// or along x with the (L+I)^-1 symbol between the forward and inverse FFTs (KIND 2).
// Persistent workgroups walk the tiles; the loads of the next tile are issued
// before the LDS stages of the current one so that HBM traffic and LDS work overlap.
// ---------------------------------------------------------------------------
// elements [FROM, TO) of the flattened (butterfly q, input m) order; the default is all of them
template <bool NT, class Tile, int N, int R, int PER, bool FULL, int FROM = 0, int TO = PER * R, class Ptr>
__device__ __forceinline__ void load_cols(float2 (&v)[PER][R], Ptr tp, int stride, int ncols, int tid) {
  // tp: first element of the tile (uniform); per-lane offsets are 32-bit
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const bool ok = bvalid<Tile, R>(q, tid);
    int i = 0, c = 0;
    if (ok) Tile::template bf<R>(tid + q * Tile::NT, i, c);
    const bool in = ok && (FULL || c < ncols);
    const int o0 = i * stride + c;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (q * R + m < FROM || q * R + m >= TO) continue;
      const int o = o0 + m * (N / R) * stride;
      if (FULL) v[q][m] = ld_g<NT>(tp + o);
      else v[q][m] = in ? ld_g<NT>(tp + o) : make_float2(0.f, 0.f);
    }
  }
}

// The persistent loop over this workgroup's tiles.  FULL: every tile has WC valid columns,
// so loads and stores need no per-lane masks (no divergent branches inside the loop).
template <int N, int KIND, bool FULL, class Ptr>
__device__ __forceinline__ void col_loop(Ptr W, Ptr Wout, const Geo& g, const Tables& tb, int64_t tile, int64_t ntiles,
                                         float2* lds, const float2* s_tw, const float* s_p2x, const float* s_p2y,
                                         const float* s_p2z, float kb2, float cim, float inv,
                                         const int32_t* act_list, ColRange rg) {
  constexpr int WC = col_wc_c(N, KIND);
  using Tile = ColTile<N, WC, col_nt_c(N, KIND)>;
  constexpr int P = plan_len(N);
  constexpr int R0 = plan_radix(N, 0, false), RL = plan_radix(N, P - 1, false);
  constexpr int PER0 = per_thread<Tile, R0>(), PERL = per_thread<Tile, RL>();
  const int tid = threadIdx.x;
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  const int CB = rg.ncb;  // column chunks walked: rg.cb0 .. rg.cb0 + rg.ncb - 1
  const int nfix = KIND == 2 ? n1 : n0;
  // W in z-lines (wz = n2) or in blocks of wz z values (w_at)
  const int wz = g.wsh < 0 ? n2 : (1 << g.wsh);
  const int stride = KIND == 2 ? n1 * wz : wz;
  // tile t = (s * nfix + fix) * CB + cb, walked with a stride of gridDim.x without divisions
  int cb = (int)(tile % CB), fix = (int)((tile / CB) % nfix), sub = (int)(tile / ((int64_t)CB * nfix));
  const int gcb = (int)(gridDim.x % CB), grest = (int)(gridDim.x / CB);
  const int gfix = grest % nfix, gsub = grest / nfix;
  // the walk runs over the iterated subdomains only (subdomain activation, Sec. 3.1): entry
  // s_ of the list, read with a scalar load so no vector load besides the tiles is in flight
  auto tile_base = [&](int s_, int fix_, int cb_) -> int64_t {
    const int sid = act_list ? cp(act_list)[__builtin_amdgcn_readfirstlane(s_)] : rg.sub0 + s_;
    const int z = (rg.cb0 + cb_) * WC;  // a tile never straddles two blocks of W
    const int64_t blk = g.wsh < 0 ? 0 : (int64_t)(z >> g.wsh) * g.wplane;
    const int zr = g.wsh < 0 ? z : (z & (wz - 1));
    return (int64_t)sid * g.sub_vox + blk + (int64_t)fix_ * (KIND == 2 ? wz : n1 * wz) + zr;
  };
  // the inverse y pass over a blocked W writes z-lines to W2 (Wout), where the z pass reads them
  const bool zl_out = KIND == 1 && g.wsh >= 0;
  const int ostride = zl_out ? n2 : stride;
  auto out_base = [&](int s_, int fix_, int cb_) -> int64_t {
    if (!zl_out) return tile_base(s_, fix_, cb_);
    const int sid = act_list ? cp(act_list)[__builtin_amdgcn_readfirstlane(s_)] : rg.sub0 + s_;
    return ((int64_t)sid * n0 + fix_) * ((int64_t)n1 * n2) + (rg.cb0 + cb_) * WC;
  };
  int c0 = (rg.cb0 + cb) * WC, ncols = min(WC, n2 - c0);
  int64_t base = tile_base(sub, fix, cb);
  float2 cur[PER0][R0];
  load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL>(cur, W + base, stride, ncols, tid);
  fft_head<Tile, N, false, KIND == 1 ? +1 : -1, PER0, R0>(cur, lds, s_tw, tid);
  // output registers of the previous tile (the FFT result that is stored)
  constexpr int PERO = KIND == 2 ? PER0 : PERL;
  constexpr int RO = KIND == 2 ? R0 : RL;
  float2 o[PERO][RO];
#pragma unroll
  for (int q = 0; q < PERO; ++q)
#pragma unroll
    for (int m = 0; m < RO; ++m) o[q][m] = make_float2(0.f, 0.f);
  for (;;) {
    const int64_t next = tile + gridDim.x;
    const bool more = next < ntiles;
    int ncb = cb + gcb, nfx = fix + gfix, nsub = sub + gsub;
    if (ncb >= CB) { ncb -= CB; ++nfx; }
    if (nfx >= nfix) { nfx -= nfix; ++nsub; }
    const int nc0 = (rg.cb0 + ncb) * WC, nncols = min(WC, n2 - nc0);
    const int64_t nbase = more ? tile_base(nsub, nfx, ncb) : base;
    float2 nxt[PER0][R0];
    // the next tile's loads are spread over the iteration (NSPL parts: before the FFT stages,
    // then between them) so the memory pipe is not idle while the current tile computes
    constexpr int NSPL = KIND == 2 ? MBS_GREEN_SPLIT : MBS_COL_SPLIT;
    constexpr int E = PER0 * R0;
    // part boundaries; the x pass with four parts also loads between its forward FFT stages
    constexpr int Q4 = (KIND == 2 && NSPL >= 4) ? E / NSPL : 0;
    constexpr int P1 = NSPL >= 2 ? Q4 + (E - Q4) / (NSPL - (Q4 ? 1 : 0)) : E;
    constexpr int P2 = NSPL >= 3 ? P1 + (E - P1) / 2 : E;
    const bool pf = MBS_COL_PREFETCH && more;
    if (pf) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL, 0, Q4 ? Q4 : P1>(nxt, W + nbase, stride, nncols, tid);
    keep_alive(o);
    if constexpr (KIND == 2) {
      float2 f[PERL][RL];
      constexpr int PL = plan_len(N);
      if constexpr (Q4 > 0 && PL > 1) {
        lds_stages<Tile, N, false, -1, 1, PL - 1>(lds, s_tw, tid);
        if (pf) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL, Q4, P1>(nxt, W + nbase, stride, nncols, tid);
        get_lds<Tile, N, RL, PERL>(lds, f, tid);
        bfly_regs<Tile, N, RL, plan_ns(N, PL - 1, false), -1, PERL>(f, s_tw, tid);
      } else {
        fft_tail<Tile, N, false, -1, PER0, R0, PERL, RL>(cur, f, lds, s_tw, tid);
      }
      // (L + I)^-1 = 1 / (1 + c (k_b^2 - |p|^2)), c = i c_im, with the 1/(n0 n1 n2) of the inverse
      const float p21 = s_p2y[fix];
#pragma unroll
      for (int q = 0; q < PERL; ++q) {
        if (!bvalid<Tile, RL>(q, tid)) continue;
        int i, c;
        Tile::template bf<RL>(tid + q * Tile::NT, i, c);
        const float p2z = s_p2z[c < ncols ? c0 + c : 0];
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          const float Pp = s_p2x[i + m * (N / RL)] + p21 + p2z;
          const float E = cim * (kb2 - Pp);
          const float den = inv * __builtin_amdgcn_rcpf(fmaf(E, E, 1.f));  // 1 ulp reciprocal
          f[q][m] = cmul(f[q][m], make_float2(den, -E * den));
        }
      }
      if (P1 < P2 && pf) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL, P1, P2>(nxt, W + nbase, stride, nncols, tid);
      fft_head<Tile, N, true, +1, PERL, RL>(f, lds, s_tw, tid);
      if (P2 < E && pf) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL, P2, E>(nxt, W + nbase, stride, nncols, tid);
      fft_tail<Tile, N, true, +1, PERL, RL, PERO, RO>(f, o, lds, s_tw, tid);
    } else {
      constexpr int PL = plan_len(N);
      constexpr int SG = KIND == 1 ? +1 : -1;
      if constexpr (PL > 1 && NSPL >= 2) {
        lds_stages<Tile, N, false, SG, 1, PL - 1>(lds, s_tw, tid);
        if (pf) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL, P1, E>(nxt, W + nbase, stride, nncols, tid);
        get_lds<Tile, N, RL, PERL>(lds, o, tid);
        bfly_regs<Tile, N, RL, plan_ns(N, PL - 1, false), SG, PERL>(o, s_tw, tid);
      } else {
        fft_tail<Tile, N, false, SG, PER0, R0, PERL, RL>(cur, o, lds, s_tw, tid);
        if (P1 < E && pf) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL, P1, E>(nxt, W + nbase, stride, nncols, tid);
      }
    }
    const auto tp = Wout + out_base(sub, fix, cb);
#pragma unroll
    for (int q = 0; q < PERO; ++q) {
      if (!bvalid<Tile, RO>(q, tid)) continue;
      int i, c;
      Tile::template bf<RO>(tid + q * Tile::NT, i, c);
      if (!FULL && c >= ncols) continue;
      const int o0 = i * ostride + c;
#pragma unroll
      for (int m = 0; m < RO; ++m) st_g<col_st_nt(KIND, N)>(tp + o0 + m * (N / RO) * ostride, o[q][m]);
    }
    if (!more) break;
    if (!MBS_COL_PREFETCH) load_cols<col_ld_nt(KIND), Tile, N, R0, PER0, FULL>(nxt, W + nbase, stride, nncols, tid);
    fft_head<Tile, N, false, KIND == 1 ? +1 : -1, PER0, R0>(nxt, lds, s_tw, tid);
#pragma unroll
    for (int q = 0; q < PER0; ++q)
#pragma unroll
      for (int m = 0; m < R0; ++m) cur[q][m] = nxt[q][m];
    tile = next;
    base = nbase;
    cb = ncb;
    fix = nfx;
    sub = nsub;
    c0 = nc0;
    ncols = nncols;
  }
}

template <int N, int KIND>
__global__ __launch_bounds__(col_nt_c(N, KIND), col_wv_c(N, KIND)) void k_col(const SlotDesc* __restrict__ tab, Geo g,
                                                                            Tables tb, int64_t ntiles, ColRange rg) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  const int32_t* act_list = nullptr;
  if (rg.nsub == g.S) {
    // every subdomain: walk the iterated ones only (subdomain activation)
    if (sd.act_list) ntiles = ntiles / g.S * sd.n_act;
    act_list = sd.act_list;
  } else if (sd.act) {
    // a block of subdomains [sub0, sub0 + nsub): a launch for idle ones does nothing
    bool any = false;
    for (int q = 0; q < rg.nsub; ++q) any = any || sub_on(sd.act, rg.sub0 + q);
    if (!any) return;
  }
  int64_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  constexpr int WC = col_wc_c(N, KIND);
  using Tile = ColTile<N, WC, col_nt_c(N, KIND)>;
  constexpr int P = plan_len(N);
  constexpr int R0 = plan_radix(N, 0, false), RL = plan_radix(N, P - 1, false);
  constexpr int PER0 = per_thread<Tile, R0>(), PERL = per_thread<Tile, RL>();
  __shared__ float2 lds[Tile::LDS];
  // twiddles and |p|^2 tables live in LDS for the whole persistent loop: the only global
  // loads in flight are then the next tile's data, so waits on them stay precise
  __shared__ float2 s_tw[N];
  __shared__ float s_p2x[KIND == 2 ? N : 1];
  __shared__ float s_p2z[KIND == 2 ? 1024 : 1];
  __shared__ float s_p2y[KIND == 2 ? 1024 : 1];
  const int tid = threadIdx.x;
  const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
  {
    const float2* twg = KIND == 2 ? tb.tw[0] : tb.tw[1];
    for (int i = tid; i < N; i += Tile::NT) s_tw[i] = twg[i];
    if constexpr (KIND == 2) {
      for (int i = tid; i < N; i += Tile::NT) s_p2x[i] = tb.p2[0][i];
      for (int i = tid; i < n2; i += Tile::NT) s_p2z[i] = tb.p2[2][i];
      for (int i = tid; i < n1; i += Tile::NT) s_p2y[i] = tb.p2[1][i];
    }
  }
  __syncthreads();
  const auto W = gp(sd.W);
  const auto Wout = KIND == 1 ? gp(sd.W2) : W;
  const float kb2 = sd.kb2, cim = sd.c_im, inv = sd.inv_vox;
  if (n2 % WC == 0)
    col_loop<N, KIND, true>(W, Wout, g, tb, tile, ntiles, lds, s_tw, s_p2x, s_p2y, s_p2z, kb2, cim, inv, act_list,
                            rg);
  else
    col_loop<N, KIND, false>(W, Wout, g, tb, tile, ntiles, lds, s_tw, s_p2x, s_p2y, s_p2z, kb2, cim, inv, act_list,
                             rg);
}


// ---------------------------------------------------------------------------
// Fused z passes over GLOBAL z-lines: one workgroup holds all P2 subdomain segments
// of a line of the global grid along z, so the z-axis edge corrections (own
// wrap-around and the neighbouring segments, Sec. 3.1) come from LDS.
//   k_fused:  inverse z FFT of iteration n, update x, residual, then w of
//             iteration n+1 and its forward z FFT (lines outside the x/y edge slabs)
//   k_wpass:  w = y + B x + edge terms and its forward z FFT (all lines at the start
//             of a solve, or only the x/y edge-slab lines after they are finished)
//   k_slabA:  finish x and d on the x/y edge-slab lines
// ---------------------------------------------------------------------------

// w = y + B x + E with a fixed operation order (E = y + corrections, summed in axis order)
__device__ __forceinline__ float2 form_w(float2 b, float2 x, float2 e) {
  return make_float2(fmaf(b.x, x.x, fmaf(-b.y, x.y, e.x)), fmaf(b.x, x.y, fmaf(b.y, x.x, e.y)));
}

// -c (C (hn - h))[a]  (low edge)  /  -c (C^T (ln - l))[a]  (high edge), with absent
// neighbours contributing zero; the same arithmetic as k_corr
__device__ __forceinline__ float2 edge_term(const float2* own, const float2* nb, bool has_nb,
                                            const float* __restrict__ C, int t, int a, bool high, float cim) {
  float2 e = make_float2(0.f, 0.f);
  for (int b = 0; b < t; ++b) {
    const float2 v = has_nb ? nb[b] : make_float2(0.f, 0.f);
    const float2 dv = csub(v, own[b]);
    const float cab = high ? C[b * t + a] : C[a * t + b];
    e.x = fmaf(cab, dv.x, e.x);
    e.y = fmaf(cab, dv.y, e.y);
  }
  return mul_negc(e, cim);
}

// x/y edge-slab lines of one column of subdomains (fixed s0, s1): region 0 = i0 in an x slab,
// region 1 = i0 outside the x slabs and i1 in a y slab
__device__ __forceinline__ int slab_line_count(const Geo& g) {
  const int in0 = g.a[0] ? g.n[0] - 2 * g.t : g.n[0];
  const int in1 = g.a[1] ? g.n[1] - 2 * g.t : g.n[1];
  return g.n[0] * g.n[1] - in0 * in1;
}
__device__ __forceinline__ void slab_line_coords(int k, const Geo& g, int& i0, int& i1) {
  const int n0 = g.n[0], n1 = g.n[1], t = g.t;
  if (g.a[0]) {
    const int r0 = 2 * t * n1;
    if (k < r0) {
      const int e = k / n1;
      i1 = k - e * n1;
      i0 = e < t ? e : n0 - 2 * t + e;
      return;
    }
    k -= r0;
    const int e = k / (2 * t), f = k - e * 2 * t;
    i0 = t + e;
    i1 = f < t ? f : n1 - 2 * t + f;
  } else {
    const int e = k / (2 * t), f = k - e * 2 * t;
    i0 = e;
    i1 = f < t ? f : n1 - 2 * t + f;
  }
}

// per-workgroup setup of segment-lines: slot l = gl * P2 + s2 holds segment s2 of global line gl
template <int L, bool SLAB_ONLY>
__device__ __forceinline__ void global_lines(const Geo& g, const SlotDesc& sd, LineInfo* info, int tid) {
  const int P2 = g.P[2];
  const int GL = L / P2;
  const int per_col = SLAB_ONLY ? slab_line_count(g) : g.n[0] * g.n[1];
  const int64_t nG = (int64_t)g.P[0] * g.P[1] * per_col;
  for (int l = tid; l < L; l += kThreads) {
    const int gl = l / P2, s2 = l - gl * P2;
    const int64_t G = (int64_t)blockIdx.x * GL + gl;
    if (G >= nG) {
      info[l].valid = 0;
      continue;
    }
    const int col = nG <= (int64_t)UINT32_MAX ? (int)((uint32_t)G / (uint32_t)per_col) : (int)(G / per_col);
    const int k = (int)(G - (int64_t)col * per_col);
    int i0, i1;
    if (SLAB_ONLY) slab_line_coords(k, g, i0, i1);
    else { i0 = k / g.n[1]; i1 = k - i0 * g.n[1]; }
    const int s = col * P2 + s2;  // col = s0 * P1 + s1
    line_info(((int64_t)s * g.n[0] + i0) * g.n[1] + i1, g, sd, info[l]);
  }
}

// any of the segment-lines this thread set up (global_lines) belongs to an iterated subdomain
template <int L>
__device__ __forceinline__ int own_lines_on(const LineInfo* info, int tid) {
  int any = 0;
  for (int l = tid; l < L; l += kThreads) any |= info[l].valid & info[l].on;
  return any;
}

// z-axis neighbour slot of segment slot l (dir = -1 low, +1 high); -1 if absent
__device__ __forceinline__ int z_neighbour(int l, int dir, const Geo& g) {
  const int P2 = g.P[2];
  if (P2 < 2) return -1;
  const int gl = l / P2, s2 = l - gl * P2;
  int sn = s2 + dir;
  if (sn < 0 || sn >= P2) {
    if (!g.periodic[2]) return -1;
    sn = (sn + P2) % P2;
  }
  return gl * P2 + sn;
}

// z edge terms of every segment-line from the edge values in zlo / zhi: ez[l][a] is the low
// edge term of element a, ez[l][t + a] the high edge term of element N - t + a
template <int L, int TM>
__device__ __forceinline__ void z_edge_terms(const float2 (*zlo)[TM], const float2 (*zhi)[TM],
                                             float2 (*ez)[2 * TM], const LineInfo* info, const Geo& g,
                                             const float* __restrict__ C, float cim, int tid) {
  const int t = g.t, tt = 2 * t;
  for (int e = tid; e < L * tt; e += kThreads) {
    const int l = e / tt, r = e - l * tt;
    if (!info[l].valid) continue;
    if (r < t) {
      const int nb = z_neighbour(l, -1, g);
      ez[l][r] = edge_term(zhi[l], nb >= 0 ? zhi[nb] : zhi[l], nb >= 0, C, t, r, false, cim);
    } else {
      const int nb = z_neighbour(l, +1, g);
      ez[l][r] = edge_term(zlo[l], nb >= 0 ? zlo[nb] : zlo[l], nb >= 0, C, t, r - t, true, cim);
    }
  }
}

// twiddles of the z FFT and the correction block C into LDS, so the FFT stages and the
// edge terms wait only on LDS
template <int N>
__device__ __forceinline__ void load_line_tables(float2* s_tw, float* s_C, const Tables& tb, const Geo& g,
                                                 int tid) {
  for (int e = tid; e < N; e += kThreads) s_tw[e] = tb.tw[2][e];
  if (g.a[2] > 0)
    for (int e = tid; e < g.t * g.t; e += kThreads) s_C[e] = tb.C[e];
}

// this thread's elements i + m N/R (butterfly q, line l) of a subdomain-major array, all loads
// issued before any is used (no branches, so the waits stay precise); lanes of an absent line,
// and with ON_ONLY of a line whose subdomain is not iterated, read line 0 instead (in bounds,
// cached, never used)
template <class Tile, int N, int R, int PER, bool ON_ONLY, class Ptr>
__device__ __forceinline__ void load_lines(float2 (&v)[PER][R], Ptr a, const LineInfo* info, int tid) {
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    int i = 0, l = 0;
    const bool ok = bvalid<Tile, R>(q, tid);
    if (ok) Tile::template bf<R>(tid + q * Tile::NT, i, l);
    const LineInfo& li = info[l];
    const int64_t base = (ok && li.valid && (!ON_ONLY || li.on)) ? li.gbase + i : i;
#pragma unroll
    for (int m = 0; m < R; ++m) v[q][m] = ld_line(a + base + m * (N / R));
  }
}

// B on this thread's elements (load_lines' element order and clamping): for a lossless medium
// one float per element (Im B) is read and Re B follows from the absorbing ramp
template <class Tile, int N, int R, int PER, bool ON_ONLY>
__device__ __forceinline__ void load_b_lines(float2 (&v)[PER][R], const SlotDesc& sd, const Geo& g,
                                             const LineInfo* info, int tid) {
  if (!sd.b_ramp) {
    load_lines<Tile, N, R, PER, ON_ONLY>(v, gp(sd.B), info, tid);
    return;
  }
  const auto Bi = gp(reinterpret_cast<const float*>(sd.B));
  // a z ramp no wider than N/R reaches only the first and last element of a butterfly: the
  // others (i + m N/R, 0 < m < R-1) are at least N/R from both ends of their segment, and a
  // segment starts at a multiple of N
  const bool narrow = sd.rw[2] <= N / R;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    int i = 0, l = 0;
    const bool ok = bvalid<Tile, R>(q, tid);
    if (ok) Tile::template bf<R>(tid + q * Tile::NT, i, l);
    const LineInfo& li = info[l];
    const int64_t base = (ok && li.valid && (!ON_ONLY || li.on)) ? li.gbase + i : i;
#pragma unroll
    for (int m = 0; m < R; ++m) v[q][m].y = ld_gf<MBS_LINE_NT != 0>(Bi + base + m * (N / R));
    if (narrow) {
      const float rb = fmaf(sd.bx_k, li.r01, 1.f);
#pragma unroll
      for (int m = 0; m < R; ++m) {
        v[q][m].x = rb;
        if (m == 0 || m == R - 1)
          v[q][m].x = fmaf(sd.bx_k, fmaxf(li.r01, ramp_axis(sd, g, 2, li.gz0 + i + m * (N / R))), 1.f);
      }
    } else {
#pragma unroll
      for (int m = 0; m < R; ++m)
        v[q][m].x = fmaf(sd.bx_k, fmaxf(li.r01, ramp_axis(sd, g, 2, li.gz0 + i + m * (N / R))), 1.f);
    }
  }
}

// t <= kMaxT: where kMaxT <= N/R only the first (m = 0) and last (m = R-1) element of a
// butterfly (i + m N/R) can lie within t of either end of its segment
template <int N, int R>
__device__ __forceinline__ bool z_edge_possible(int m) {
  return kMaxT > N / R || m == 0 || m == R - 1;
}

// z edge values of this thread's elements to LDS (first t to zlo, last t to zhi); with ON_ONLY
// a line whose subdomain is not iterated has the edge values of its field, zero
template <class Tile, int N, int R, int PER, int TM, bool ON_ONLY>
__device__ __forceinline__ void put_z_edges(const float2 (&v)[PER][R], float2 (*zlo)[TM],
                                            float2 (*zhi)[TM], const LineInfo* info, int t, int tid) {
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    if (!bvalid<Tile, R>(q, tid)) continue;
    int i, l;
    Tile::template bf<R>(tid + q * Tile::NT, i, l);
    if (!info[l].valid) continue;
    const bool zero = ON_ONLY && !info[l].on;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if (!z_edge_possible<N, R>(m)) continue;
      const int j = i + m * (N / R);
      const float2 e = zero ? make_float2(0.f, 0.f) : v[q][m];
      if (j < t) zlo[l][j] = e;
      if (j >= N - t) zhi[l][j - (N - t)] = e;
    }
  }
}

// z edge term of element j of segment-line l (zero away from the edges)
template <int N, int TM>
__device__ __forceinline__ float2 z_edge_at(const float2 (*ez)[2 * TM], int l, int j, int t) {
  if (j < t) return ez[l][j];
  if (j >= N - t) return ez[l][j - (N - 2 * t)];
  return make_float2(0.f, 0.f);
}

template <int N, bool SLAB_ONLY>
__global__ __launch_bounds__(kThreads) void k_wpass(const SlotDesc* __restrict__ tab, Geo g, Tables tb) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  constexpr int L = lines_per_wg_c(N);
  using Tile = LineTile<N, L>;
  constexpr int P = plan_len(N);
  constexpr int R0 = plan_radix(N, 0, false), RL = plan_radix(N, P - 1, false);
  constexpr int PER0 = per_thread<Tile, R0>(), PERL = per_thread<Tile, RL>();
  __shared__ float2 lds[Tile::LDS];
  __shared__ LineInfo info[L];
  constexpr int TM = kMaxT < N / 2 ? kMaxT : N / 2;  // t <= min(kMaxT, N / 2)
  __shared__ float2 zlo[L][TM], zhi[L][TM], ez[L][2 * TM];
  __shared__ float2 s_tw[N];
  __shared__ float s_C[kMaxT * kMaxT];
  const int tid = threadIdx.x;
  global_lines<L, SLAB_ONLY>(g, sd, info, tid);
  load_line_tables<N>(s_tw, s_C, tb, g, tid);
  // W is written only on lines of iterated subdomains; a workgroup with none has nothing to do
  if (!__syncthreads_or(own_lines_on<L>(info, tid))) return;
  const int t = g.t;
  const bool zc = g.a[2] > 0;
  const float cim = sd.c_im;
  const auto E0 = gp(sd.slab[0][2]);
  const auto E1 = gp(sd.slab[1][2]);
  const auto Y = gp(sd.ybox);
  const auto W = gp(sd.W);
  // the edge-slab pass reads only iterated lines; the pass over every line (start of a solve,
  // or lines of newly activated subdomains) reads all of them: x is zero where not iterated
  float2 xv[PER0][R0], bv[PER0][R0];
  load_lines<Tile, N, R0, PER0, SLAB_ONLY>(xv, gp(sd.x), info, tid);
  load_b_lines<Tile, N, R0, PER0, SLAB_ONLY>(bv, sd, g, info, tid);
  if (zc) {
    put_z_edges<Tile, N, R0, PER0, TM, SLAB_ONLY>(xv, zlo, zhi, info, t, tid);
    __syncthreads();
    z_edge_terms<L, TM>(zlo, zhi, ez, info, g, s_C, cim, tid);
    __syncthreads();
  }
  float2 v[PER0][R0];
#pragma unroll
  for (int q = 0; q < PER0; ++q) {
    int i = 0, l = 0;
    const bool ok = bvalid<Tile, R0>(q, tid);
    if (ok) Tile::template bf<R0>(tid + q * Tile::NT, i, l);
    const LineInfo& li = info[l];
#pragma unroll
    for (int m = 0; m < R0; ++m) {
      const int j = i + m * (N / R0);
      float2 w = make_float2(0.f, 0.f);
      if (ok && li.valid && li.on) {
        float2 e = make_float2(0.f, 0.f);
        if (j >= li.jlo && j < li.jhi) e = Y[li.ybase + j];
        if (li.e0 >= 0) e = cadd(e, E0[li.e0 + j]);
        if (li.e1 >= 0) e = cadd(e, E1[li.e1 + j]);
        if (zc && z_edge_possible<N, R0>(m)) e = cadd(e, z_edge_at<N, TM>(ez, l, j, t));
        w = form_w(bv[q][m], xv[q][m], e);
      }
      v[q][m] = w;
    }
  }
  float2 o[PERL][RL];
  fft_tile<Tile, N, false, -1>(v, o, lds, s_tw, tid);
#pragma unroll
  for (int q = 0; q < PERL; ++q) {
    if (!bvalid<Tile, RL>(q, tid)) continue;
    int i, l;
    Tile::template bf<RL>(tid + q * Tile::NT, i, l);
    if (!info[l].valid || !info[l].on) continue;
    const auto p = W + (info[l].wbase + w_off(i, g));
#pragma unroll
    for (int m = 0; m < RL; ++m) st_line(p + w_off(m * (N / RL), g), o[q][m]);
  }
}

template <int N>
__global__ __launch_bounds__(kThreads, 4) void k_fused(const SlotDesc* __restrict__ tab, Geo g, Tables tb) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  constexpr int L = lines_per_wg_c(N);
  using Tile = LineTile<N, L>;
  constexpr int P = plan_len(N);
  // inverse with the reversed radix order ends in the forward plan's first radix, so the
  // inverse outputs a thread holds are exactly the forward stage-0 inputs it needs
  constexpr int RI = plan_radix(N, 0, true), R0 = plan_radix(N, 0, false), RL = plan_radix(N, P - 1, false);
  constexpr int PI = per_thread<Tile, RI>(), PER0 = per_thread<Tile, R0>(), PERL = per_thread<Tile, RL>();
  __shared__ float2 lds[Tile::LDS];
  __shared__ LineInfo info[L];
  constexpr int TM = kMaxT < N / 2 ? kMaxT : N / 2;  // t <= min(kMaxT, N / 2)
  __shared__ float2 zlo[L][TM], zhi[L][TM], ez[L][2 * TM];
  __shared__ float2 s_tw[N];
  __shared__ float s_C[kMaxT * kMaxT];
  __shared__ double red[kThreads / 64];
  __shared__ int any_plain;
  const int tid = threadIdx.x;
  global_lines<L, false>(g, sd, info, tid);
  load_line_tables<N>(s_tw, s_C, tb, g, tid);
  if (tid == 0) any_plain = 0;
  if (!__syncthreads_or(own_lines_on<L>(info, tid))) {
    // every line here belongs to a subdomain that is not iterated (activation)
    if (tid == 0) gp(sd.part_main)[blockIdx.x] = 0.0;
    return;
  }
  const int t = g.t;
  const bool zc = g.a[2] > 0;
  const float cim = sd.c_im, alpha = sd.alpha;
  const auto X = gp(sd.x);
  const auto W = gp(sd.W);
  // every global read of the tile is issued here: v of iteration n (the inverse y pass's output,
  // in z-lines), x_n and B
  float2 vin[PI][RI], xv[PER0][R0], bv[PER0][R0];
  load_lines<Tile, N, RI, PI, true>(vin, gp(sd.W2), info, tid);
  load_lines<Tile, N, R0, PER0, true>(xv, X, info, tid);
  load_b_lines<Tile, N, R0, PER0, true>(bv, sd, g, info, tid);
  float2 u[PER0][R0];
  fft_tile<Tile, N, true, +1>(vin, u, lds, s_tw, tid);
  // u = x - v; the z edge terms of u
#pragma unroll
  for (int q = 0; q < PER0; ++q)
#pragma unroll
    for (int m = 0; m < R0; ++m) u[q][m] = csub(xv[q][m], u[q][m]);
  if (zc) {
    put_z_edges<Tile, N, R0, PER0, TM, true>(u, zlo, zhi, info, t, tid);
    __syncthreads();
    z_edge_terms<L, TM>(zlo, zhi, ez, info, g, s_C, cim, tid);
    __syncthreads();
  }
  const auto U0 = gp(sd.slab[0][1]);
  const auto U1 = gp(sd.slab[1][1]);
  double acc = 0.0;
  bool plain_here = false;
#pragma unroll
  for (int q = 0; q < PER0; ++q) {
    int i = 0, l = 0;
    const bool ok = bvalid<Tile, R0>(q, tid);
    if (ok) Tile::template bf<R0>(tid + q * Tile::NT, i, l);
    const LineInfo& li = info[l];
    if (!(ok && li.valid && li.on)) continue;
    const bool slab = li.e0 >= 0 || li.e1 >= 0;
#pragma unroll
    for (int m = 0; m < R0; ++m) {
      const int j = i + m * (N / R0);
      const int64_t gi = li.gbase + j;
      float2 d = cmul(bv[q][m], u[q][m]);
      if (zc && z_edge_possible<N, R0>(m)) d = cadd(d, z_edge_at<N, TM>(ez, l, j, t));
      const float2 xn = make_float2(fmaf(-alpha, d.x, xv[q][m].x), fmaf(-alpha, d.y, xv[q][m].y));
      st_line(X + gi, xn);
      if (slab) {
        // x/y edge-slab line: its x/y corrections come later (k_slabA); keep the partial d in W
        st_line(W + (li.wbase + w_off(i, g) + w_off(m * (N / R0), g)), d);
        if (li.e0 >= 0) U0[li.e0 + j] = u[q][m];
        if (li.e1 >= 0) U1[li.e1 + j] = u[q][m];
      } else {
        acc += norm2d(d);
      }
      xv[q][m] = xn;
    }
    plain_here |= !slab;
  }
  if (plain_here) any_plain = 1;
  __syncthreads();
  // next iteration's w on the lines that are complete
  if (any_plain) {
    const auto Y = gp(sd.ybox);
    if (zc) {
      put_z_edges<Tile, N, R0, PER0, TM, true>(xv, zlo, zhi, info, t, tid);
      __syncthreads();
      z_edge_terms<L, TM>(zlo, zhi, ez, info, g, s_C, cim, tid);
      __syncthreads();
    }
    float2 v[PER0][R0];
#pragma unroll
    for (int q = 0; q < PER0; ++q) {
      int i = 0, l = 0;
      const bool ok = bvalid<Tile, R0>(q, tid);
      if (ok) Tile::template bf<R0>(tid + q * Tile::NT, i, l);
      const LineInfo& li = info[l];
      const bool plain = ok && li.valid && li.on && li.e0 < 0 && li.e1 < 0;
#pragma unroll
      for (int m = 0; m < R0; ++m) {
        const int j = i + m * (N / R0);
        float2 w = make_float2(0.f, 0.f);
        if (plain) {
          float2 e = make_float2(0.f, 0.f);
          if (j >= li.jlo && j < li.jhi) e = Y[li.ybase + j];
          if (zc && z_edge_possible<N, R0>(m)) e = cadd(e, z_edge_at<N, TM>(ez, l, j, t));
          w = form_w(bv[q][m], xv[q][m], e);
        }
        v[q][m] = w;
      }
    }
    float2 o[PERL][RL];
    fft_tile<Tile, N, false, -1>(v, o, lds, s_tw, tid);
#pragma unroll
    for (int q = 0; q < PERL; ++q) {
      if (!bvalid<Tile, RL>(q, tid)) continue;
      int i, l;
      Tile::template bf<RL>(tid + q * Tile::NT, i, l);
      const LineInfo& li = info[l];
      if (!li.valid || !li.on || li.e0 >= 0 || li.e1 >= 0) continue;
      const auto p = W + (li.wbase + w_off(i, g));
#pragma unroll
      for (int m = 0; m < RL; ++m) st_line(p + w_off(m * (N / RL), g), o[q][m]);
    }
  }
  const double ssum = block_sum(acc, red);
  if (tid == 0) gp(sd.part_main)[blockIdx.x] = ssum;
}

// finish the x/y edge-slab lines: d = d_partial + Eu_0 + Eu_1, x -= alpha (Eu_0 + Eu_1),
// edge slabs X_0 / X_1 of the new iterate, residual partial sums
__global__ __launch_bounds__(kThreads) void k_slabA(const SlotDesc* __restrict__ tab, Geo g) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  __shared__ double red[kThreads / 64];
  // each subdomain has its own run of blocks: the subdomain follows from the block index, the
  // line and z index from one 32-bit division (edge-slab voxels of one subdomain: below 2^31)
  const int n2 = g.n[2], t = g.t;
  const int per_sub = slab_line_count(g) * n2;
  const int bps = (per_sub + kThreads - 1) / kThreads;
  const int s = (int)blockIdx.x / bps;
  const int r = ((int)blockIdx.x - s * bps) * kThreads + (int)threadIdx.x;
  double acc = 0.0;
  if (r < per_sub && sub_on(sd.act, s)) {
    const int k = r / n2;
    const int j = r - k * n2;
    int i0, i1;
    slab_line_coords(k, g, i0, i1);
    const int64_t line = ((int64_t)s * g.n[0] + i0) * g.n[1] + i1;
    const int64_t gi = line * n2 + j;
    float2 esum = make_float2(0.f, 0.f);
    // edge-slab buffers of one axis hold S 2 t n_p n_q <= S n0 n1 n2 < 2^31 values
    int a0 = -1, a1 = -1;
    if (g.a[0] && (i0 < t || i0 >= g.n[0] - t)) {
      const int side = i0 < t ? 0 : 1, aa = side ? i0 - (g.n[0] - t) : i0;
      a0 = ((s * 2 + side) * t + aa) * (g.n[1] * n2) + i1 * n2 + j;
      esum = cadd(esum, gp(sd.slab[0][3])[a0]);
    }
    if (g.a[1] && (i1 < t || i1 >= g.n[1] - t)) {
      const int side = i1 < t ? 0 : 1, aa = side ? i1 - (g.n[1] - t) : i1;
      a1 = ((s * 2 + side) * t + aa) * (g.n[0] * n2) + i0 * n2 + j;
      esum = cadd(esum, gp(sd.slab[1][3])[a1]);
    }
    const float2 d = cadd(gp(sd.W)[w_at(w_line_base(s, i0, i1, g), j, g)], esum);
    const float2 xv = gp(sd.x)[gi];
    const float2 xn = make_float2(fmaf(-sd.alpha, esum.x, xv.x), fmaf(-sd.alpha, esum.y, xv.y));
    gp(sd.x)[gi] = xn;
    if (a0 >= 0) gp(sd.slab[0][0])[a0] = xn;
    if (a1 >= 0) gp(sd.slab[1][0])[a1] = xn;
    acc = norm2d(d);
  }
  const double ssum = block_sum(acc, red);
  if (threadIdx.x == 0) gp(sd.part_face)[blockIdx.x] = ssum;
}

// ---------------------------------------------------------------------------
// Subdomain activation (Sec. 3.1, end): the field an iterated neighbour transfers into a
// subdomain that is not iterated.  There x = 0, so its edge terms are exactly the transfer:
// along x and y they are the corrections of the iterate the slab pass already wrote
// (E = -c C h of the neighbour), along z they are formed here from the neighbours' t edge
// values.  Workgroup b of subdomain s writes the partial sum of |E|^2 over its share of the
// faces to xfer[s * kXferBlocks + b] (zero for iterated subdomains).
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(kThreads) void k_xfer(const SlotDesc* __restrict__ tab, Geo g,
                                                   const float* __restrict__ C) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.xfer == nullptr || sd.st->done == kIdle) return;
  __shared__ double red[kThreads / 64];
  const int s = blockIdx.x / kXferBlocks, b = blockIdx.x - s * kXferBlocks;
  const int64_t step = (int64_t)kXferBlocks * kThreads;
  double acc = 0.0;
  if (!sub_on(sd.act, s)) {
    for (int d = 0; d < 2; ++d) {
      if (!g.a[d]) continue;
      const int64_t plane = d == 0 ? (int64_t)g.n[1] * g.n[2] : (int64_t)g.n[0] * g.n[2];
      const int64_t cnt = 2 * (int64_t)T * plane;  // both sides of subdomain s
      const auto E = gp(sd.slab[d][2]) + (int64_t)s * cnt;
      for (int64_t e = (int64_t)b * kThreads + threadIdx.x; e < cnt; e += step) {
        const float2 v = E[e];
        acc += norm2d(v);
      }
    }
    const int P2 = g.P[2];
    if (g.a[2] == 2) {
      const int s2 = s % P2;
      int slo = s2 - 1, shi = s2 + 1;
      if (slo < 0) slo = g.periodic[2] ? P2 - 1 : -1;
      if (shi >= P2) shi = g.periodic[2] ? 0 : -1;
      if (slo >= 0) slo = s - s2 + slo;
      if (shi >= 0) shi = s - s2 + shi;
      const bool lo_on = slo >= 0 && sub_on(sd.act, slo);
      const bool hi_on = shi >= 0 && sub_on(sd.act, shi);
      const int n2 = g.n[2];
      const int64_t nl = (int64_t)g.n[0] * g.n[1];
      const double c2 = (double)sd.c_im * (double)sd.c_im;
      const auto X = gp(sd.x);
      for (int64_t k = (int64_t)b * kThreads + threadIdx.x; k < nl; k += step) {
        if (lo_on) {  // last T values of the lower neighbour enter through the low edge
          float2 h[T];
#pragma unroll
          for (int j = 0; j < T; ++j) h[j] = X[((int64_t)slo * nl + k) * n2 + (n2 - T) + j];
#pragma unroll
          for (int a = 0; a < T; ++a) {
            float2 e = make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < T; ++j) {
              e.x = fmaf(C[a * T + j], h[j].x, e.x);
              e.y = fmaf(C[a * T + j], h[j].y, e.y);
            }
            acc += c2 * norm2d(e);
          }
        }
        if (hi_on) {  // first T values of the upper neighbour enter through the high edge
          float2 l[T];
#pragma unroll
          for (int j = 0; j < T; ++j) l[j] = X[((int64_t)shi * nl + k) * n2 + j];
#pragma unroll
          for (int a = 0; a < T; ++a) {
            float2 e = make_float2(0.f, 0.f);
#pragma unroll
            for (int j = 0; j < T; ++j) {
              e.x = fmaf(C[j * T + a], l[j].x, e.x);
              e.y = fmaf(C[j * T + a], l[j].y, e.y);
            }
            acc += c2 * norm2d(e);
          }
        }
      }
    }
  }
  const double sum = block_sum(acc, red);
  if (threadIdx.x == 0) sd.xfer[blockIdx.x] = sum;
}

// ---------------------------------------------------------------------------
// edge corrections along one axis: for each line, from the first t (l) and
// last t (h) values of the subdomain and its neighbours,
//   E_lo[a] = -c (C (h_{s-1} - h_s))[a],   E_hi[a] = -c (C^T (l_{s+1} - l_s))[a]
// with absent neighbours contributing zero (Sec. 3 and Sec. 3.1 steps 1-5).
// which = 0: X -> Ex (iterate), 1: U -> Eu (u = x - v).
// ---------------------------------------------------------------------------
template <int T>
__global__ __launch_bounds__(kThreads) void k_corr(const SlotDesc* __restrict__ tab, Geo g,
                                                   const float* __restrict__ C, int d, int which) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  const int64_t plane = d == 0 ? (int64_t)g.n[1] * g.n[2]
                               : (d == 1 ? (int64_t)g.n[0] * g.n[2] : (int64_t)g.n[0] * g.n[1]);
  const int64_t L = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (L >= (int64_t)g.S * plane) return;
  const int s = (int)(L / plane);
  const int64_t pq = L - (int64_t)s * plane;
  int sc[3];
  sc[2] = s % g.P[2];
  sc[1] = (s / g.P[2]) % g.P[1];
  sc[0] = s / (g.P[2] * g.P[1]);
  const int Pd = g.P[d];
  const bool cyc = g.periodic[d] && Pd >= 2;
  const bool has_lo = Pd >= 2 && (sc[d] > 0 || cyc);
  const bool has_hi = Pd >= 2 && (sc[d] < Pd - 1 || cyc);
  const int mul = d == 0 ? g.P[1] * g.P[2] : (d == 1 ? g.P[2] : 1);
  const int s_lo = s + (((sc[d] - 1 + Pd) % Pd) - sc[d]) * mul;
  const int s_hi = s + (((sc[d] + 1) % Pd) - sc[d]) * mul;
  const auto src = gp(sd.slab[d][which == 0 ? 0 : 1]);
  const auto dst = gp(sd.slab[d][which == 0 ? 2 : 3]);
  float2 dh[T], dl[T];
#pragma unroll
  for (int b = 0; b < T; ++b) {
    const float2 h = src[(((int64_t)s * 2 + 1) * T + b) * plane + pq];
    const float2 l = src[(((int64_t)s * 2 + 0) * T + b) * plane + pq];
    const float2 hn = has_lo ? src[(((int64_t)s_lo * 2 + 1) * T + b) * plane + pq] : make_float2(0.f, 0.f);
    const float2 ln = has_hi ? src[(((int64_t)s_hi * 2 + 0) * T + b) * plane + pq] : make_float2(0.f, 0.f);
    dh[b] = csub(hn, h);
    dl[b] = csub(ln, l);
  }
  const float cim = sd.c_im;
#pragma unroll
  for (int a = 0; a < T; ++a) {
    float2 elo = make_float2(0.f, 0.f), ehi = make_float2(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const float cab = C[a * T + b];
      const float cba = C[b * T + a];
      elo.x = fmaf(cab, dh[b].x, elo.x);
      elo.y = fmaf(cab, dh[b].y, elo.y);
      ehi.x = fmaf(cba, dl[b].x, ehi.x);
      ehi.y = fmaf(cba, dl[b].y, ehi.y);
    }
    dst[(((int64_t)s * 2 + 0) * T + a) * plane + pq] = mul_negc(elo, cim);
    dst[(((int64_t)s * 2 + 1) * T + a) * plane + pq] = mul_negc(ehi, cim);
  }
}

// ---------------------------------------------------------------------------
// face update over the union of the edge slabs (disjoint regions per axis):
//   d = B u + sum Eu,  x -= alpha sum Eu,  X slabs <- x,  partial sum |d|^2
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_face(const SlotDesc* __restrict__ tab, Geo g) {
  const SlotDesc sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  __shared__ double red[kThreads / 64];
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double acc = 0.0;
  if (gid < (int64_t)g.S * g.face_vox) {
    const int s = (int)(gid / g.face_vox);
    int64_t r = gid - (int64_t)s * g.face_vox;
    int reg = 0;
    while (r >= g.reg_count[reg]) {
      r -= g.reg_count[reg];
      ++reg;
    }
    const int e2 = (int)(r % g.reg_ext[reg][2]);
    r /= g.reg_ext[reg][2];
    const int e1 = (int)(r % g.reg_ext[reg][1]);
    const int e0 = (int)(r / g.reg_ext[reg][1]);
    int e[3] = {e0, e1, e2};
    int i[3];
    const int t = g.t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k == reg) i[k] = e[k] < t ? e[k] : g.n[k] - 2 * t + e[k];
      else i[k] = e[k] + g.reg_off[reg][k];
    }
    float2 esum = make_float2(0.f, 0.f), u = make_float2(0.f, 0.f);
    int64_t addr[3] = {-1, -1, -1};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (g.a[k] == 0) continue;
      int side, aa;
      if (i[k] < t) { side = 0; aa = i[k]; }
      else if (i[k] >= g.n[k] - t) { side = 1; aa = i[k] - (g.n[k] - t); }
      else continue;
      const int p = k == 0 ? i[1] : i[0];
      const int q = k == 2 ? i[1] : i[2];
      const int dq = k == 2 ? g.n[1] : g.n[2];
      const int64_t plane = k == 0 ? (int64_t)g.n[1] * g.n[2]
                                   : (k == 1 ? (int64_t)g.n[0] * g.n[2] : (int64_t)g.n[0] * g.n[1]);
      const int64_t ad = (((int64_t)s * 2 + side) * t + aa) * plane + (int64_t)p * dq + q;
      addr[k] = ad;
      esum = cadd(esum, gp(sd.slab[k][3])[ad]);
      u = gp(sd.slab[k][1])[ad];
    }
    const int64_t gi = (((int64_t)s * g.n[0] + i[0]) * g.n[1] + i[1]) * g.n[2] + i[2];
    float2 bv;
    if (sd.b_ramp) {
      const int c2 = s % g.P[2], c1 = (s / g.P[2]) % g.P[1], c0 = s / (g.P[2] * g.P[1]);
      const float rr = fmaxf(fmaxf(ramp_axis(sd, g, 0, c0 * g.n[0] + i[0]), ramp_axis(sd, g, 1, c1 * g.n[1] + i[1])),
                             ramp_axis(sd, g, 2, c2 * g.n[2] + i[2]));
      bv = make_float2(fmaf(sd.bx_k, rr, 1.f), gp(reinterpret_cast<const float*>(sd.B))[gi]);
    } else {
      bv = gp(sd.B)[gi];
    }
    const float2 bu = cmul(bv, u);
    const float2 dd = cadd(bu, esum);
    const float2 xv = gp(sd.x)[gi];
    const float2 xn = make_float2(fmaf(-sd.alpha, esum.x, xv.x), fmaf(-sd.alpha, esum.y, xv.y));
    gp(sd.x)[gi] = xn;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (addr[k] >= 0) gp(sd.slab[k][0])[addr[k]] = xn;
    acc = norm2d(dd);
  }
  const double ssum = block_sum(acc, red);
  if (threadIdx.x == 0) gp(sd.part_face)[blockIdx.x] = ssum;
}

// ---------------------------------------------------------------------------
// residual norm in two fixed-order stages: kReduceBlocks workgroups sum contiguous
// ranges of the partials, then one workgroup per slot sums those and applies the
// relative residual and stop test (Sec. 3.1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_reduce1(const SlotDesc* __restrict__ tab, int64_t n_main,
                                                      int64_t n_face) {
  const SlotDesc& sd = tab[blockIdx.y];
  if (sd.st->done != kRunning) return;
  __shared__ double red[kThreads / 64];
  const int64_t total = n_main + n_face;
  const int64_t chunk = (total + kReduceBlocks - 1) / kReduceBlocks;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < total ? lo + chunk : total;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads)
    acc += i < n_main ? gp(sd.part_main)[i] : gp(sd.part_face)[i - n_main];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) gp(sd.part_red)[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_reduce2(const SlotDesc* __restrict__ tab) {
  const SlotDesc& sd = tab[blockIdx.x];
  SlotState* st = sd.st;
  if (st->done != kRunning) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < kReduceBlocks; i += 64) acc += sd.part_red[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (threadIdx.x != 0) return;
  const double rho = sqrt(acc);
  st->rho = rho;
  if (st->probe) {
    st->done = isfinite(rho) ? kConverged : kNonFinite;
    return;
  }
  const int it = st->iter;
  if (it == 0 && !(st->rho_ref > 0.0)) st->rho_ref = rho;
  const double eps = st->rho_ref > 0.0 ? rho / st->rho_ref : 0.0;
  if (it < kHistCap) sd.hist[it] = eps;
  st->iter = it + 1;
  st->eps = eps;
  if (!isfinite(rho)) st->done = kNonFinite;
  else if (eps < st->tol) st->done = kConverged;
  else if (it > 0 && st->eps_prev > 1e-5 && eps > st->eps_prev * 1.01) st->done = kDiverged;
  else if (it + 1 >= st->max_iter) st->done = kMaxIter;
  st->eps_prev = eps;
}

// ---------------------------------------------------------------------------
// set-up kernels (FP64 medium statistics, operator diagonal, source, layout)
// ---------------------------------------------------------------------------
struct Int3 { int32_t v[3]; };

__device__ __forceinline__ void global_coords(int64_t v, const Geo& g, int& g0, int& g1, int& g2) {
  g2 = (int)(v % g.N[2]);
  const int64_t r = v / g.N[2];
  g1 = (int)(r % g.N[1]);
  g0 = (int)(r / g.N[1]);
}

__device__ __forceinline__ int64_t local_index(int g0, int g1, int g2, const Geo& g) {
  const int s0 = g0 / g.n[0], s1 = g1 / g.n[1], s2 = g2 / g.n[2];
  const int i0 = g0 - s0 * g.n[0], i1 = g1 - s1 * g.n[1], i2 = g2 - s2 * g.n[2];
  const int s = (s0 * g.P[1] + s1) * g.P[2] + s2;
  return (((int64_t)s * g.n[0] + i0) * g.n[1] + i1) * g.n[2] + i2;
}

// Im(n^2) of the absorbing layer: linear ramp over the outermost W voxels of each side,
// maximum over axes
__device__ __forceinline__ double ramp_at(int g0, int g1, int g2, const Geo& g, const Int3& w,
                                          double rmax) {
  const int gc[3] = {g0, g1, g2};
  double r = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int W = w.v[d];
    if (W <= 0) continue;
    const int i = gc[d];
    if (i < W) r = fmax(r, rmax * (double)(W - i) / (double)W);
    if (i >= g.N[d] - W) r = fmax(r, rmax * (double)(i - (g.N[d] - W) + 1) / (double)W);
  }
  return r;
}

__device__ __forceinline__ void wavenumber_sq(const float2* n, int64_t v, const Geo& g, double k0sq,
                                              const Int3& w, double rmax, double& re, double& im,
                                              bool& finite) {
  const float2 nv = n[v];
  const double nr = nv.x, ni = nv.y;
  finite = isfinite(nr) && isfinite(ni);
  int g0, g1, g2;
  global_coords(v, g, g0, g1, g2);
  const double n2r = nr * nr - ni * ni;
  const double n2i = nr * ni + ni * nr + ramp_at(g0, g1, g2, g, w, rmax);
  re = k0sq * n2r;
  im = k0sq * n2i;
}

__global__ __launch_bounds__(kThreads) void k_medium_stats(const float2* __restrict__ n, Geo g,
                                                           double k0sq, Int3 w, double rmax,
                                                           MediumStats* part) {
  __shared__ double smin[kThreads], smax[kThreads], simin[kThreads], snf[kThreads], snim[kThreads];
  double mn = INFINITY, mx = -INFINITY, imn = INFINITY, nf = 0.0, nim = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.vox;
       v += (int64_t)gridDim.x * kThreads) {
    double re, im;
    bool fin;
    wavenumber_sq(n, v, g, k0sq, w, rmax, re, im, fin);
    if (!fin) { nf += 1.0; continue; }
    mn = fmin(mn, re);
    mx = fmax(mx, re);
    imn = fmin(imn, im);
    nim = fmax(nim, fabs((double)n[v].y));
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  simin[threadIdx.x] = imn;
  snf[threadIdx.x] = nf;
  snim[threadIdx.x] = nim;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
      simin[threadIdx.x] = fmin(simin[threadIdx.x], simin[threadIdx.x + off]);
      snf[threadIdx.x] += snf[threadIdx.x + off];
      snim[threadIdx.x] = fmax(snim[threadIdx.x], snim[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x].re_min = smin[0];
    part[blockIdx.x].re_max = smax[0];
    part[blockIdx.x].im_min = simin[0];
    part[blockIdx.x].nonfinite = snf[0];
    part[blockIdx.x].nim_max = snim[0];
  }
}

__global__ __launch_bounds__(kThreads) void k_medium_kmax(const float2* __restrict__ n, Geo g,
                                                          double k0sq, Int3 w, double rmax,
                                                          double kb2, double* part) {
  __shared__ double sm[kThreads];
  double mx = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.vox;
       v += (int64_t)gridDim.x * kThreads) {
    double re, im;
    bool fin;
    wavenumber_sq(n, v, g, k0sq, w, rmax, re, im, fin);
    mx = fmax(mx, hypot(re - kb2, im));
  }
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// B = 1 - c (k^2 - k_b^2), c = i c_im, written subdomain-major
__global__ __launch_bounds__(kThreads) void k_medium_B(const float2* __restrict__ n, Geo g, double k0sq,
                                                       Int3 w, double rmax, double kb2, double c_im,
                                                       float2* __restrict__ B, int compact) {
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.vox;
       v += (int64_t)gridDim.x * kThreads) {
    double re, im;
    bool fin;
    wavenumber_sq(n, v, g, k0sq, w, rmax, re, im, fin);
    const double zr = re - kb2, zi = im;
    int g0, g1, g2;
    global_coords(v, g, g0, g1, g2);
    if (compact)  // lossless medium: Im B only (Re B = 1 + c_im k0^2 ramp is rebuilt where it is used)
      reinterpret_cast<float*>(B)[local_index(g0, g1, g2, g)] = (float)(-c_im * zr);
    else
      B[local_index(g0, g1, g2, g)] = make_float2((float)fma(c_im, zi, 1.0), (float)(-c_im * zr));
  }
}

__global__ __launch_bounds__(kThreads) void k_source_bbox(const float2* __restrict__ S, Geo g,
                                                          int32_t* bbox) {
  __shared__ int32_t sm[7][kThreads];
  int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {-1, -1, -1}, bad = 0;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.vox;
       v += (int64_t)gridDim.x * kThreads) {
    const float2 s = S[v];
    if (!(isfinite(s.x) && isfinite(s.y))) {
      bad = 1;
      continue;
    }
    if (s.x == 0.f && s.y == 0.f) continue;
    int gc[3];
    global_coords(v, g, gc[0], gc[1], gc[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], gc[d]);
      hi[d] = max(hi[d], gc[d]);
    }
  }
  for (int d = 0; d < 3; ++d) {
    sm[d][threadIdx.x] = lo[d];
    sm[3 + d][threadIdx.x] = hi[d];
  }
  sm[6][threadIdx.x] = bad;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      for (int d = 0; d < 3; ++d) {
        sm[d][threadIdx.x] = min(sm[d][threadIdx.x], sm[d][threadIdx.x + off]);
        sm[3 + d][threadIdx.x] = max(sm[3 + d][threadIdx.x], sm[3 + d][threadIdx.x + off]);
      }
      sm[6][threadIdx.x] |= sm[6][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (sm[6][0]) atomicOr(&bbox[6], 1);
    if (sm[3][0] >= 0) {
      for (int d = 0; d < 3; ++d) {
        atomicMin(&bbox[d], sm[d][0]);
        atomicMax(&bbox[3 + d], sm[3 + d][0]);
      }
    }
  }
}

// y = -c S on the bounding box, box-local C-order
__global__ __launch_bounds__(kThreads) void k_source_fill(const float2* __restrict__ S, Geo g, Int3 lo,
                                                          Int3 ext, double c_im, float2* __restrict__ y) {
  const int64_t nb = (int64_t)ext.v[0] * ext.v[1] * ext.v[2];
  const float cim = (float)c_im;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < nb;
       v += (int64_t)gridDim.x * kThreads) {
    const int b2 = (int)(v % ext.v[2]);
    const int64_t r = v / ext.v[2];
    const int b1 = (int)(r % ext.v[1]);
    const int b0 = (int)(r / ext.v[1]);
    const int64_t gv = ((int64_t)(b0 + lo.v[0]) * g.N[1] + (b1 + lo.v[1])) * g.N[2] + (b2 + lo.v[2]);
    y[v] = mul_negc(S[gv], cim);
  }
}

__global__ __launch_bounds__(kThreads) void k_scatter(const float2* __restrict__ f, Geo g,
                                                      float2* __restrict__ x) {
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.vox;
       v += (int64_t)gridDim.x * kThreads) {
    int g0, g1, g2;
    global_coords(v, g, g0, g1, g2);
    x[local_index(g0, g1, g2, g)] = f[v];
  }
}

__global__ __launch_bounds__(kThreads) void k_gather(const float2* __restrict__ x, Geo g,
                                                     float2* __restrict__ f) {
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < g.vox;
       v += (int64_t)gridDim.x * kThreads) {
    int g0, g1, g2;
    global_coords(v, g, g0, g1, g2);
    f[v] = x[local_index(g0, g1, g2, g)];
  }
}

__global__ __launch_bounds__(kThreads) void k_zero(float2* __restrict__ p, int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kThreads)
    p[v] = make_float2(0.f, 0.f);
}

// copy the edge slabs of the iterate (which = 0 -> X) of one slot from x
__global__ __launch_bounds__(kThreads) void k_extract(const SlotDesc* __restrict__ tab, int slot, Geo g,
                                                     int d) {
  const SlotDesc sd = tab[slot];
  const int t = g.t;
  const int64_t plane = d == 0 ? (int64_t)g.n[1] * g.n[2]
                               : (d == 1 ? (int64_t)g.n[0] * g.n[2] : (int64_t)g.n[0] * g.n[1]);
  const int64_t total = (int64_t)g.S * 2 * t * plane;
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < total;
       v += (int64_t)gridDim.x * kThreads) {
    const int64_t pq = v % plane;
    const int64_t r = v / plane;
    const int aa = (int)(r % t);
    const int side = (int)((r / t) % 2);
    const int s = (int)(r / (2 * t));
    const int pos = side ? g.n[d] - t + aa : aa;
    const int dq = d == 2 ? g.n[1] : g.n[2];
    const int p = (int)(pq / dq);
    const int q = (int)(pq % dq);
    int i[3];
    i[d] = pos;
    if (d == 0) { i[1] = p; i[2] = q; }
    else if (d == 1) { i[0] = p; i[2] = q; }
    else { i[0] = p; i[1] = q; }
    const int64_t gi = (((int64_t)s * g.n[0] + i[0]) * g.n[1] + i[1]) * g.n[2] + i[2];
    sd.slab[d][0][v] = sd.x[gi];
  }
}

// small stream-ordered control writes (values travel as kernel arguments)
__global__ void k_put_state(SlotState* dst, SlotState v) {
  if (threadIdx.x == 0) *dst = v;
}
__global__ void k_put_desc(SlotDesc* dst, SlotDesc v) {
  if (threadIdx.x == 0) *dst = v;
}
struct Int8 { int32_t v[8]; };
__global__ void k_put_i32x8(int32_t* dst, Int8 v) {
  if (threadIdx.x < 8) dst[threadIdx.x] = v.v[threadIdx.x];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t put_state(SlotState* dst, const SlotState& v, hipStream_t s) {
  hipLaunchKernelGGL(k_put_state, dim3(1), dim3(64), 0, s, dst, v);
  return hipGetLastError();
}
hipError_t put_desc(SlotDesc* dst, const SlotDesc& v, hipStream_t s) {
  hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, dst, v);
  return hipGetLastError();
}
hipError_t put_i32x8(int32_t* dst, const int32_t* v, hipStream_t s) {
  Int8 w;
  for (int i = 0; i < 8; ++i) w.v[i] = v[i];
  hipLaunchKernelGGL(k_put_i32x8, dim3(1), dim3(64), 0, s, dst, w);
  return hipGetLastError();
}

int lines_per_wg(int n) { return lines_per_wg_c(n); }

#define MBS_FOR_EACH_N(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool fft_size_supported(int n) {
  switch (n) {
#define MBS_CASE(NN) case NN:
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    return true;
    default:
      return false;
  }
}

static inline unsigned grid_1d(int64_t work, int64_t cap = 1 << 20) {
  int64_t b = (work + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

int64_t last_pass_blocks(const Geo& g) {
  const int64_t lines = (int64_t)g.S * g.n[0] * g.n[1];
  const int L = lines_per_wg_c(g.n[2]);
  return (lines + L - 1) / L;
}

int64_t face_blocks(const Geo& g) {
  return ((int64_t)g.S * g.face_vox + kThreads - 1) / kThreads;
}

hipError_t launch_first_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                             hipStream_t s) {
  dim3 grid((unsigned)last_pass_blocks(g), nslots);
  switch (g.n[2]) {
#define MBS_CASE(NN) \
  case NN: hipLaunchKernelGGL(k_first<NN>, grid, dim3(kThreads), 0, s, tab, g, tb); break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_last_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                            hipStream_t s) {
  dim3 grid((unsigned)last_pass_blocks(g), nslots);
  switch (g.n[2]) {
#define MBS_CASE(NN) \
  case NN: hipLaunchKernelGGL(k_last<NN>, grid, dim3(kThreads), 0, s, tab, g, tb); break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// workgroups of a column kernel resident per compute unit (registers and LDS), queried once
template <int NN, int KIND>
static int col_resident_per_cu() {
  static const int v = [] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_col<NN, KIND>),
                                                     col_nt_c(NN, KIND), 0) != hipSuccess || nb < 1)
      nb = 1;
    return nb;
  }();
  return v;
}

// persistent grid: every resident workgroup slot of the device, at most one per tile
static inline unsigned persistent_grid(int64_t ntiles, const Geo& g, int per_cu) {
  const int64_t cap = (int64_t)per_cu * (g.cus > 0 ? g.cus : 256);
  return (unsigned)(ntiles < cap ? ntiles : cap);
}

template <int NN, int KIND>
static void launch_col(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, hipStream_t s,
                       ColRange rg) {
  constexpr int WC = col_wc_c(NN, KIND);
  const int fix = KIND == 2 ? g.n[1] : g.n[0];
  if (rg.ncb <= 0) {
    rg.sub0 = 0;
    rg.nsub = g.S;
    rg.cb0 = 0;
    rg.ncb = (g.n[2] + WC - 1) / WC;
  }
  const int64_t ntiles = (int64_t)rg.nsub * fix * rg.ncb;
  dim3 grid(persistent_grid(ntiles, g, col_resident_per_cu<NN, KIND>()), nslots);
  hipLaunchKernelGGL((k_col<NN, KIND>), grid, dim3(col_nt_c(NN, KIND)), 0, s, tab, g, tb, ntiles, rg);
}

int col_chunk_width(int n, int kind) {
  return kind == 2 ? (n >= MBS_GREEN_MIN_N && n <= 512 ? MBS_GREEN_WC : cols_per_tile_c(n)) : cols_per_tile_c(n);
}

// occupancy queries of the plan's column kernels, made before any stream capture
void prepare_launches(const Geo& g) {
  switch (g.n[1]) {
#define MBS_CASE(NN)                 \
  case NN:                           \
    (void)col_resident_per_cu<NN, 0>(); \
    (void)col_resident_per_cu<NN, 1>(); \
    break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      break;
  }
  switch (g.n[0]) {
#define MBS_CASE(NN) \
  case NN: (void)col_resident_per_cu<NN, 2>(); break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      break;
  }
}

hipError_t launch_mid_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                           int inverse, hipStream_t s, ColRange rg) {
  switch (g.n[1]) {
#define MBS_CASE(NN)                                              \
  case NN:                                                        \
    if (inverse) launch_col<NN, 1>(tab, nslots, g, tb, s, rg);    \
    else launch_col<NN, 0>(tab, nslots, g, tb, s, rg);            \
    break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_green_pass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb,
                             hipStream_t s, ColRange rg) {
  switch (g.n[0]) {
#define MBS_CASE(NN) \
  case NN: launch_col<NN, 2>(tab, nslots, g, tb, s, rg); break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_corr(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, int which,
                       hipStream_t s, int axis_mask) {
  for (int d = 0; d < 3; ++d) {
    if (g.a[d] == 0 || !(axis_mask & (1 << d))) continue;
    const int64_t plane = d == 0 ? (int64_t)g.n[1] * g.n[2]
                                 : (d == 1 ? (int64_t)g.n[0] * g.n[2] : (int64_t)g.n[0] * g.n[1]);
    const int64_t lines = (int64_t)g.S * plane;
    dim3 grid((unsigned)((lines + kThreads - 1) / kThreads), nslots);
    switch (g.t) {
#define MBS_T(TT) \
  case TT: hipLaunchKernelGGL(k_corr<TT>, grid, dim3(kThreads), 0, s, tab, g, tb.C, d, which); break;
      MBS_T(1) MBS_T(2) MBS_T(3) MBS_T(4) MBS_T(5) MBS_T(6) MBS_T(7) MBS_T(8)
      MBS_T(9) MBS_T(10) MBS_T(11) MBS_T(12) MBS_T(13) MBS_T(14) MBS_T(15) MBS_T(16)
#undef MBS_T
      default:
        return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int host_slab_line_count(const Geo& g) {
  const int in0 = g.a[0] ? g.n[0] - 2 * g.t : g.n[0];
  const int in1 = g.a[1] ? g.n[1] - 2 * g.t : g.n[1];
  return g.n[0] * g.n[1] - in0 * in1;
}

bool fusion_supported(const Geo& g) { return lines_per_wg_c(g.n[2]) % g.P[2] == 0; }

int64_t slabA_blocks(const Geo& g) {
  return (int64_t)g.S * (((int64_t)host_slab_line_count(g) * g.n[2] + kThreads - 1) / kThreads);
}

hipError_t launch_fused(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, hipStream_t s) {
  dim3 grid((unsigned)last_pass_blocks(g), nslots);
  switch (g.n[2]) {
#define MBS_CASE(NN) \
  case NN: hipLaunchKernelGGL(k_fused<NN>, grid, dim3(kThreads), 0, s, tab, g, tb); break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_wpass(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, int slab_only,
                        hipStream_t s) {
  const int L = lines_per_wg_c(g.n[2]);
  const int64_t per_col = slab_only ? host_slab_line_count(g) : (int64_t)g.n[0] * g.n[1];
  const int64_t segs = (int64_t)g.P[0] * g.P[1] * per_col * g.P[2];
  if (segs == 0) return hipSuccess;
  dim3 grid((unsigned)((segs + L - 1) / L), nslots);
  switch (g.n[2]) {
#define MBS_CASE(NN)                                                                              \
  case NN:                                                                                        \
    if (slab_only) hipLaunchKernelGGL((k_wpass<NN, true>), grid, dim3(kThreads), 0, s, tab, g, tb);  \
    else hipLaunchKernelGGL((k_wpass<NN, false>), grid, dim3(kThreads), 0, s, tab, g, tb);           \
    break;
    MBS_FOR_EACH_N(MBS_CASE)
#undef MBS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_slabA(const SlotDesc* tab, int nslots, const Geo& g, hipStream_t s) {
  const int64_t nb = slabA_blocks(g);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slabA, dim3((unsigned)nb, nslots), dim3(kThreads), 0, s, tab, g);
  return hipGetLastError();
}

hipError_t launch_face(const SlotDesc* tab, int nslots, const Geo& g, hipStream_t s) {
  dim3 grid((unsigned)face_blocks(g), nslots);
  hipLaunchKernelGGL(k_face, grid, dim3(kThreads), 0, s, tab, g);
  return hipGetLastError();
}

hipError_t launch_reduce(const SlotDesc* tab, int nslots, const Geo& g, int64_t n_main,
                         int64_t n_face, hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_reduce1, dim3(kReduceBlocks, nslots), dim3(kThreads), 0, s, tab, n_main, n_face);
  hipLaunchKernelGGL(k_reduce2, dim3(nslots), dim3(64), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_xfer(const SlotDesc* tab, int nslots, const Geo& g, const Tables& tb, hipStream_t s) {
  dim3 grid((unsigned)(g.S * kXferBlocks), nslots);
  switch (g.t) {
#define MBS_T(TT) \
  case TT: hipLaunchKernelGGL(k_xfer<TT>, grid, dim3(kThreads), 0, s, tab, g, tb.C); break;
    MBS_T(1) MBS_T(2) MBS_T(3) MBS_T(4) MBS_T(5) MBS_T(6) MBS_T(7) MBS_T(8)
    MBS_T(9) MBS_T(10) MBS_T(11) MBS_T(12) MBS_T(13) MBS_T(14) MBS_T(15) MBS_T(16)
#undef MBS_T
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int64_t setup_blocks(const Geo& g) { return grid_1d(g.vox, 4096); }

hipError_t launch_medium_stats(const float2* n, const Geo& g, double k0sq, const int32_t* width,
                               double ramp_max, MediumStats* partials, int64_t nblocks,
                               hipStream_t s) {
  Int3 w{{width[0], width[1], width[2]}};
  hipLaunchKernelGGL(k_medium_stats, dim3((unsigned)nblocks), dim3(kThreads), 0, s, n, g, k0sq, w,
                     ramp_max, partials);
  return hipGetLastError();
}

hipError_t launch_medium_kmax(const float2* n, const Geo& g, double k0sq, const int32_t* width,
                              double ramp_max, double kb2, double* partials, int64_t nblocks,
                              hipStream_t s) {
  Int3 w{{width[0], width[1], width[2]}};
  hipLaunchKernelGGL(k_medium_kmax, dim3((unsigned)nblocks), dim3(kThreads), 0, s, n, g, k0sq, w,
                     ramp_max, kb2, partials);
  return hipGetLastError();
}

hipError_t launch_medium_B(const float2* n, const Geo& g, double k0sq, const int32_t* width,
                           double ramp_max, double kb2, double c_im, float2* B, int compact, hipStream_t s) {
  Int3 w{{width[0], width[1], width[2]}};
  hipLaunchKernelGGL(k_medium_B, dim3(grid_1d(g.vox)), dim3(kThreads), 0, s, n, g, k0sq, w, ramp_max,
                     kb2, c_im, B, compact);
  return hipGetLastError();
}

hipError_t launch_source_bbox(const float2* S, const Geo& g, int32_t* bbox, hipStream_t s) {
  hipLaunchKernelGGL(k_source_bbox, dim3(grid_1d(g.vox, 8192)), dim3(kThreads), 0, s, S, g, bbox);
  return hipGetLastError();
}

hipError_t launch_source_fill(const float2* S, const Geo& g, const int32_t* lo, const int32_t* ext,
                              double c_im, float2* ybox, hipStream_t s) {
  Int3 l{{lo[0], lo[1], lo[2]}}, e{{ext[0], ext[1], ext[2]}};
  const int64_t nb = (int64_t)ext[0] * ext[1] * ext[2];
  hipLaunchKernelGGL(k_source_fill, dim3(grid_1d(nb)), dim3(kThreads), 0, s, S, g, l, e, c_im, ybox);
  return hipGetLastError();
}

hipError_t launch_scatter(const float2* field, const Geo& g, float2* x, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(grid_1d(g.vox)), dim3(kThreads), 0, s, field, g, x);
  return hipGetLastError();
}

hipError_t launch_gather(const float2* x, const Geo& g, float2* field, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(grid_1d(g.vox)), dim3(kThreads), 0, s, x, g, field);
  return hipGetLastError();
}

hipError_t launch_zero(float2* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero, dim3(grid_1d(n)), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_extract_slabs(const SlotDesc* tab, int slot, const Geo& g, int which,
                                hipStream_t s) {
  (void)which;
  for (int d = 0; d < 3; ++d) {
    if (g.a[d] == 0) continue;
    const int64_t plane = d == 0 ? (int64_t)g.n[1] * g.n[2]
                                 : (d == 1 ? (int64_t)g.n[0] * g.n[2] : (int64_t)g.n[0] * g.n[1]);
    const int64_t total = (int64_t)g.S * 2 * g.t * plane;
    hipLaunchKernelGGL(k_extract, dim3(grid_1d(total)), dim3(kThreads), 0, s, tab, slot, g, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mbs
