// Streaming-bandwidth probe: what plain HBM streams reach on this GPU, as the
// yardstick for the vertex step's measured traffic rate.  Standalone program
// (no library code): 1 GiB of FP64 data, 16-byte loads, each configuration
// timed with HIP events over 20 launches after 3 warm-up launches.
//
//   read, grid-stride     every thread walks the array with the grid's stride
//                         (all waves inside one sliding window)
//   read, one pass        one 16-byte load per thread, n / 256 blocks
//   read, block ranges    each block streams its own contiguous range, in
//                         4 KiB steps, from NS separate arrays (NS = 1, 3);
//                         with 30 KiB of dynamic LDS per block the occupancy
//                         is that of the LDS-staged vertex kernel (5 blocks of
//                         4 waves per CU); 8,921 blocks as in its 1025^2 launch
//   copy, grid-stride     0.5 GiB read + 0.5 GiB written
//
// Output: one markdown table row per configuration.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define PROBE_CHECK(x)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));               \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

namespace {

// The sums are kept alive by a store that never happens (the data are zeros).
__global__ void k_read_stride(const double2* __restrict__ a, size_t n, double* __restrict__ out) {
  double s = 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = a[i];
    s += v.x + v.y;
  }
  if (s == 1.0) out[blockIdx.x] = s;
}

__global__ void k_read_once(const double2* __restrict__ a, size_t n, double* __restrict__ out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    const double2 v = a[i];
    s = v.x + v.y;
  }
  if (s == 1.0) out[blockIdx.x] = s;
}

// Block b reads elements [b * per, (b + 1) * per) of each of NS arrays of
// n_per_stream elements (b * per + per <= n_per_stream by construction).
template <int NS>
__global__ void __launch_bounds__(256) k_read_ranges(const double2* __restrict__ a, size_t n_per_stream, int per,
                                                     double* __restrict__ out) {
  const size_t base = (size_t)blockIdx.x * per;
  double s = 0.0;
  for (int i = 0; i < per; i += 256) {
    const int j = i + (int)threadIdx.x;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const double2 v = j < per ? a[k * n_per_stream + base + j] : make_double2(0.0, 0.0);
      s += v.x + v.y;
    }
  }
  if (s == 1.0) out[blockIdx.x] = s;
}

__global__ void k_copy(const double2* __restrict__ a, double2* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <class Launch>
double time_us(Launch&& launch) {
  hipEvent_t e0, e1;
  PROBE_CHECK(hipEventCreate(&e0));
  PROBE_CHECK(hipEventCreate(&e1));
  for (int r = 0; r < 3; ++r) launch();
  PROBE_CHECK(hipEventRecord(e0, nullptr));
  const int reps = 20;
  for (int r = 0; r < reps; ++r) launch();
  PROBE_CHECK(hipEventRecord(e1, nullptr));
  PROBE_CHECK(hipEventSynchronize(e1));
  PROBE_CHECK(hipGetLastError());
  float ms = 0.f;
  PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
  PROBE_CHECK(hipEventDestroy(e0));
  PROBE_CHECK(hipEventDestroy(e1));
  return 1e3 * ms / reps;
}

void row(const char* kind, long grid, int lds_kb, int streams, double us, double bytes) {
  std::printf("| %s | %ld | %d | %d | %.1f | %.3f |\n", kind, grid, lds_kb, streams, us, bytes / (us * 1e-6) / 1e12);
  std::fflush(stdout);
}

}  // namespace

int main() {
  const size_t bytes = size_t(1) << 30;
  const size_t n = bytes / sizeof(double2);
  double2 *a = nullptr, *b = nullptr;
  double* out = nullptr;
  const size_t out_n = size_t(1) << 20;   // >= every grid below
  PROBE_CHECK(hipMalloc(&a, bytes));
  PROBE_CHECK(hipMalloc(&b, bytes / 2));
  PROBE_CHECK(hipMalloc(&out, out_n * sizeof(double)));
  PROBE_CHECK(hipMemset(a, 0, bytes));
  PROBE_CHECK(hipMemset(b, 0, bytes / 2));
  hipDeviceProp_t prop;
  PROBE_CHECK(hipGetDeviceProperties(&prop, 0));
  std::printf("device: %s, %d CUs; 1 GiB per read configuration\n\n", prop.name, prop.multiProcessorCount);
  std::printf("| kind | blocks | dynamic LDS (KiB) | streams | us | TB/s |\n|---|---|---|---|---|---|\n");

  for (int grid : {1024, 2048, 4096, 8192}) {
    const double us = time_us([&] { k_read_stride<<<grid, 256>>>(a, n, out); });
    row("read, grid-stride", grid, 0, 1, us, (double)bytes);
  }
  {
    const int grid = (int)(n / 256);   // 262,144 blocks
    const double us = time_us([&] { k_read_once<<<grid, 256>>>(a, n, out); });
    row("read, one pass", grid, 0, 1, us, (double)bytes);
  }
  for (int lds_kb : {0, 30}) {
    for (int ns : {1, 3}) {
      const int blocks = 8921;
      const size_t nps = n / ns;
      const int per = (int)(nps / blocks);
      const double moved = (double)per * blocks * ns * sizeof(double2);
      const size_t lds = (size_t)lds_kb * 1024;
      const double us = time_us([&] {
        if (ns == 1)
          k_read_ranges<1><<<blocks, 256, lds>>>(a, nps, per, out);
        else
          k_read_ranges<3><<<blocks, 256, lds>>>(a, nps, per, out);
      });
      row("read, block ranges", blocks, lds_kb, ns, us, moved);
    }
  }
  {
    const int grid = 2048;
    const double us = time_us([&] { k_copy<<<grid, 256>>>(a, b, n / 2); });
    row("copy, grid-stride", grid, 0, 1, us, (double)bytes);
  }
  PROBE_CHECK(hipFree(a));
  PROBE_CHECK(hipFree(b));
  PROBE_CHECK(hipFree(out));
  return 0;
}
