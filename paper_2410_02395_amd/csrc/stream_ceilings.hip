// Streaming rates of the device's HBM for the read:write mixes of the solver's kernels.
//
// A stand-alone measurement program (not part of the library): plain element-wise streams over
// 2 GiB arrays, each timed with HIP events as the best of 10 launches, printed one JSON object
// per line.  The mixes are those of the iteration: 1:1 (the FFT passes, in place), 3:2 (the
// fused z pass: W, x, B in; x, W out), and pure reads and writes for reference.  The rates bound
// what the solver's kernels can reach on the same part; they say nothing about the algorithm.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                           \
  do {                                                                                     \
    hipError_t err_ = (x);                                                                 \
    if (err_ != hipSuccess) {                                                              \
      fprintf(stderr, "stream_ceilings: %s at line %d\n", hipGetErrorString(err_), __LINE__); \
      exit(1);                                                                             \
    }                                                                                      \
  } while (0)

namespace {

typedef float v4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4 ld(const v4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(v4* p, v4 v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// one 8-byte element per thread (the access width of the solver's kernels); n elements
__global__ __launch_bounds__(256) void k_copy8(const float2* __restrict__ a, float2* __restrict__ b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// 16-byte elements, U per thread, one trip over the array (grid covers it); n16 elements
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy16(const v4* __restrict__ a, v4* __restrict__ b, long n16) {
  const long base = (long)blockIdx.x * blockDim.x * U + threadIdx.x;
  v4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long i = base + (long)u * blockDim.x;
    v[u] = i < n16 ? ld<NT>(a + i) : v4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long i = base + (long)u * blockDim.x;
    if (i < n16) st<NT>(b + i, v[u]);
  }
}

// three reads, two writes per element
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_r3w2(const v4* __restrict__ a, const v4* __restrict__ b,
                                              const v4* __restrict__ c, v4* __restrict__ d,
                                              v4* __restrict__ e, long n16) {
  const long base = (long)blockIdx.x * blockDim.x * U + threadIdx.x;
  v4 va[U], vb[U], vc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long i = base + (long)u * blockDim.x;
    const bool ok = i < n16;
    va[u] = ok ? ld<NT>(a + i) : v4{0.f, 0.f, 0.f, 0.f};
    vb[u] = ok ? ld<NT>(b + i) : v4{0.f, 0.f, 0.f, 0.f};
    vc[u] = ok ? ld<NT>(c + i) : v4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long i = base + (long)u * blockDim.x;
    if (i < n16) {
      st<NT>(d + i, va[u] + vb[u] * vc[u]);
      st<NT>(e + i, va[u] - vc[u]);
    }
  }
}

// reads with a grid-stride loop over a persistent grid; one partial sum per thread
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_read(const v4* __restrict__ a, float* __restrict__ out, long n16) {
  const long stride = (long)gridDim.x * blockDim.x * U;
  float s = 0.f;
  for (long base = (long)blockIdx.x * blockDim.x * U + threadIdx.x; base < n16; base += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long i = base + (long)u * blockDim.x;
      if (i < n16) {
        const v4 v = ld<NT>(a + i);
        s += v.x + v.y + v.z + v.w;
      }
    }
  }
  out[(long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int U>
__global__ __launch_bounds__(256) void k_write(v4* __restrict__ b, long n16, float val) {
  const long base = (long)blockIdx.x * blockDim.x * U + threadIdx.x;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long i = base + (long)u * blockDim.x;
    if (i < n16) b[i] = v4{val, val, val, val};
  }
}

}  // namespace

int main() {
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  const long bytes = 2L << 30;  // per array
  const long n16 = bytes / 16;
  v4 *a, *b, *c, *d, *e;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMalloc(&c, bytes));
  CHECK(hipMalloc(&d, bytes));
  CHECK(hipMalloc(&e, bytes));
  const int read_grid = cus * 8;
  float* partial;
  CHECK(hipMalloc(&partial, (size_t)read_grid * 256 * sizeof(float)));
  for (v4* p : {a, b, c, d, e}) CHECK(hipMemset(p, 0, bytes));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  auto blocks = [&](int per_thread) { return (unsigned)((n16 + 256L * per_thread - 1) / (256L * per_thread)); };
  auto run = [&](const char* name, const char* mix, double moved, auto launch) {
    launch();
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int r = 0; r < 10; ++r) {
      CHECK(hipEventRecord(e0));
      launch();
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) best = ms;
    }
    CHECK(hipGetLastError());
    printf("{\"kernel\": \"%s\", \"mix\": \"%s\", \"bytes\": %.0f, \"ms\": %.4f, \"gbps\": %.1f}\n", name, mix, moved,
           best, moved / (best * 1e-3) / 1e9);
    fflush(stdout);
  };
  run("hipMemcpyAsync device to device", "read 1, write 1", 2.0 * bytes,
      [&] { CHECK(hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, 0)); });
  run("copy, 8 B per thread", "read 1, write 1", 2.0 * bytes, [&] {
    k_copy8<<<dim3((unsigned)((bytes / 8 + 255) / 256)), 256>>>((const float2*)a, (float2*)b, bytes / 8);
  });
  run("copy, 16 B per thread", "read 1, write 1", 2.0 * bytes,
      [&] { k_copy16<1, false><<<blocks(1), 256>>>(a, b, n16); });
  run("copy, 4 x 16 B per thread, nontemporal", "read 1, write 1", 2.0 * bytes,
      [&] { k_copy16<4, true><<<blocks(4), 256>>>(a, b, n16); });
  run("three reads, two writes, 2 x 16 B per thread", "read 3, write 2", 5.0 * bytes,
      [&] { k_r3w2<2, false><<<blocks(2), 256>>>(a, b, c, d, e, n16); });
  run("three reads, two writes, 2 x 16 B per thread, nontemporal", "read 3, write 2", 5.0 * bytes,
      [&] { k_r3w2<2, true><<<blocks(2), 256>>>(a, b, c, d, e, n16); });
  run("read, persistent grid, nontemporal", "read 1", 1.0 * bytes,
      [&] { k_read<4, true><<<read_grid, 256>>>(a, partial, n16); });
  run("write, 4 x 16 B per thread", "write 1", 1.0 * bytes,
      [&] { k_write<4><<<blocks(4), 256>>>(b, n16, 1.0f); });
  for (v4* p : {a, b, c, d, e}) CHECK(hipFree(p));
  CHECK(hipFree(partial));
  return 0;
}
