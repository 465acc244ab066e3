// Standalone profiling driver for rocprofv3 (no Python, no torch): applies
// M_pc^+ M_pc through the C ABI on a unit-link lattice (memory traffic does
// not depend on the link values), or runs a plain copy kernel of known size
// to calibrate the FETCH_SIZE / WRITE_SIZE counters.
//
//   hdcg_prof H <X> <Y> <Z> <T> <Ls> <c128|c64|bf16> <reps> [nrhs] [shape]
//   hdcg_prof copy|copy4|read <MiB> <reps> [grid]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../../include/hdcg.h"

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e = (x);                                                       \
    if (e != hipSuccess) {                                                    \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));             \
      return 1;                                                               \
    }                                                                         \
  } while (0)
#define ACHECK(x)                                                             \
  do {                                                                        \
    int r = (x);                                                              \
    if (r < 0) {                                                              \
      std::fprintf(stderr, "%s -> %d: %s\n", #x, r, dwf_last_error());        \
      return 1;                                                               \
    }                                                                         \
  } while (0)

__global__ void copy_kernel(const double4* __restrict__ x, double4* __restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// copy with four 32-byte loads in flight per thread before the stores, and
// non-temporal stores (n a multiple of 4 * grid * block is not required)
__global__ void copy4_kernel(const double4* __restrict__ x, double4* __restrict__ y, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = x[i + k * stride];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      typedef double d4 __attribute__((ext_vector_type(4)));
      const d4 w = {v[k].x, v[k].y, v[k].z, v[k].w};
      __builtin_nontemporal_store(w, reinterpret_cast<d4*>(y + i + k * stride));
    }
  }
  for (; i < n; i += stride) y[i] = x[i];
}

// streaming read: one partial sum per thread (n / (grid * block) loads each)
__global__ void read_kernel(const double4* __restrict__ x, double* __restrict__ y, size_t n) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double4 v = x[i];
    s += v.x + v.y + v.z + v.w;
  }
  y[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  if (!std::strcmp(argv[1], "copy") || !std::strcmp(argv[1], "read") || !std::strcmp(argv[1], "copy4")) {
    // hdcg_prof copy|copy4|read <MiB> <reps> [grid]: plain copy (copy4: four
    // loads in flight per thread, non-temporal stores) or streaming read of MiB
    const bool rd = !std::strcmp(argv[1], "read"), c4 = !std::strcmp(argv[1], "copy4");
    const size_t mib = argc > 2 ? std::atol(argv[2]) : 1024;
    const int reps = argc > 3 ? std::atoi(argv[3]) : 3;
    const int grid = argc > 4 ? std::atoi(argv[4]) : 4096;
    const size_t n = mib * 1024 * 1024 / sizeof(double4);
    double4 *x, *y;
    double* part;
    CHECK(hipMalloc(&x, n * sizeof(double4)));
    CHECK(hipMalloc(&y, n * sizeof(double4)));
    CHECK(hipMalloc(&part, (size_t)grid * 256 * sizeof(double)));
    CHECK(hipMemset(x, 0, n * sizeof(double4)));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) {
      if (rd)
        hipLaunchKernelGGL(read_kernel, dim3(grid), dim3(256), 0, 0, x, part, n);
      else if (c4)
        hipLaunchKernelGGL(copy4_kernel, dim3(grid), dim3(256), 0, 0, x, y, n);
      else
        hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, 0, x, y, n);
    }
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    const double bytes = (double)n * 32 * (rd ? 1 : 2);
    std::printf("%s %zu MiB x %d grid %d (bytes per launch read %zu write %zu)  %.4f ms/launch  %.1f GB/s\n",
                argv[1], mib, reps, grid, n * 32, rd ? (size_t)0 : n * 32, ms / reps,
                bytes / (ms / reps * 1e-3) / 1e9);
    return 0;
  }
  if (!std::strcmp(argv[1], "sweep")) {
    // hdcg_prof sweep X Y Z T Ls prec(c128|c64|bf16) reps shape1 shape2 ...
    // (shape = "bx,by,bz,bt[,remap,lds_kb,nt,morton,phases,rg]", see dwf_set_hop_shape)
    int dims[4] = {std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), std::atoi(argv[5])};
    const int Ls = std::atoi(argv[6]);
    const int prec = !std::strcmp(argv[7], "c64") ? DWF_C64 : (!std::strcmp(argv[7], "bf16") ? DWF_BF16 : DWF_C128);
    const int reps = std::atoi(argv[8]);
    const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
    std::vector<double> U(V * 4 * 9 * 2, 0.0);
    for (size_t l = 0; l < V * 4; ++l)
      for (int a = 0; a < 3; ++a) U[(l * 9 + a * 4) * 2] = 1.0;
    void* dU;
    CHECK(hipMalloc(&dU, U.size() * sizeof(double)));
    CHECK(hipMemcpy(dU, U.data(), U.size() * sizeof(double), hipMemcpyHostToDevice));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int a = 9; a < argc; ++a) {
      int shape[10] = {2, 2, 1, 1, 1, 0, 0, 1, 0, 1};
      if (std::sscanf(argv[a], "%d,%d,%d,%d,%d,%d,%d,%d,%d,%d", &shape[0], &shape[1], &shape[2], &shape[3], &shape[4],
                      &shape[5], &shape[6], &shape[7], &shape[8], &shape[9]) < 4) {
        std::fprintf(stderr, "bad shape %s\n", argv[a]);
        return 2;
      }
      dwf_op_t op;
      ACHECK(dwf_create(&op, dims, Ls, 1.8, 0.01, dU, nullptr, nullptr));
      ACHECK(dwf_set_hop_shape(op, shape));
      size_t bytes = 0;
      ACHECK(dwf_field_bytes(op, prec, 1, &bytes));
      void *x, *y;
      CHECK(hipMalloc(&x, bytes));
      CHECK(hipMalloc(&y, bytes));
      CHECK(hipMemset(x, 0, bytes));
      for (int r = 0; r < 3; ++r) ACHECK(mpc_dag_mpc_apply(op, y, x, prec, 1, nullptr));
      CHECK(hipEventRecord(e0, nullptr));
      for (int r = 0; r < reps; ++r) ACHECK(mpc_dag_mpc_apply(op, (r & 1) ? x : y, (r & 1) ? y : x, prec, 1, nullptr));
      CHECK(hipEventRecord(e1, nullptr));
      CHECK(hipEventSynchronize(e1));
      float ms = 0;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      // field bytes per complex (16-bit fields: 4) and link bytes per complex
      // (complex64 links with 16-bit fields)
      const double half = (double)V / 2 * Ls * 12;
      const double cb = prec == DWF_C128 ? 16 : (prec == DWF_C64 ? 8 : 4), gb = prec == DWF_C128 ? 16 : 8;
      const double by = 10 * half * cb + 4.0 * V * 36 * gb;
      std::printf("tile %-14s %s %dx%dx%dx%d Ls=%d  %.4f ms/H  %.1f GB/s\n", argv[a], argv[7], dims[0], dims[1],
                  dims[2], dims[3], Ls, ms / reps, by / (ms / reps * 1e-3) / 1e9);
      std::fflush(stdout);
      CHECK(hipFree(x));
      CHECK(hipFree(y));
      ACHECK(dwf_destroy(op));
    }
    return 0;
  }
  if (argc < 9) return 2;
  int dims[4] = {std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4]), std::atoi(argv[5])};
  const int Ls = std::atoi(argv[6]);
  const int prec = !std::strcmp(argv[7], "c64") ? DWF_C64 : (!std::strcmp(argv[7], "bf16") ? DWF_BF16 : DWF_C128);
  const int reps = std::atoi(argv[8]);
  const int nrhs = argc > 9 ? std::atoi(argv[9]) : 1;
  // optional fixed launch shape "bx,by,bz,bt[,remap,lds_kb,nt,morton,phases,rg]" (else autotuned)
  int shape[10] = {2, 2, 1, 1, 1, 0, 0, 1, 0, 1};
  const bool fixed = argc > 10 && std::sscanf(argv[10], "%d,%d,%d,%d,%d,%d,%d,%d,%d,%d", &shape[0], &shape[1],
                                               &shape[2], &shape[3], &shape[4], &shape[5], &shape[6], &shape[7],
                                               &shape[8], &shape[9]) >= 4;
  const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
  std::vector<double> U(V * 4 * 9 * 2, 0.0);
  for (size_t l = 0; l < V * 4; ++l)
    for (int a = 0; a < 3; ++a) U[(l * 9 + a * 4) * 2] = 1.0;
  void* dU;
  CHECK(hipMalloc(&dU, U.size() * sizeof(double)));
  CHECK(hipMemcpy(dU, U.data(), U.size() * sizeof(double), hipMemcpyHostToDevice));
  dwf_op_t op;
  ACHECK(dwf_create(&op, dims, Ls, 1.8, 0.01, dU, nullptr, nullptr));
  if (fixed) ACHECK(dwf_set_hop_shape(op, shape));
  size_t bytes = 0;
  ACHECK(dwf_field_bytes(op, prec, nrhs, &bytes));
  void *x, *y;
  CHECK(hipMalloc(&x, bytes));
  CHECK(hipMalloc(&y, bytes));
  std::vector<unsigned char> h(bytes);
  for (size_t i = 0; i < bytes; ++i) h[i] = (unsigned char)((i * 2654435761u) >> 24) & 0x3f;
  CHECK(hipMemcpy(x, h.data(), bytes, hipMemcpyHostToDevice));
  for (int r = 0; r < reps; ++r) {
    ACHECK(mpc_dag_mpc_apply(op, y, x, prec, nrhs, nullptr));
    ACHECK(mpc_dag_mpc_apply(op, x, y, prec, nrhs, nullptr));
  }
  CHECK(hipDeviceSynchronize());
  ACHECK(dwf_destroy(op));
  std::printf("H %s %dx%dx%dx%d Ls=%d nrhs=%d x %d\n", argv[7], dims[0], dims[1], dims[2], dims[3], Ls, nrhs, 2 * reps);
  return 0;
}
