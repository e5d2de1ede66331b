// Small kernels: fills and the interface sum over duplicated DoFs.
#include "tmf_internal.h"

namespace tmf {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t n, T v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

// A DoF on a face, edge or vertex shared by several macro-tets has one copy
// per macro; after the macro-local applies every copy holds a partial sum.
// One thread per duplicate group adds the copies in ascending slot order and
// writes the total to all of them (deterministic).
template <typename T>
__global__ __launch_bounds__(256) void k_interface(GroupArgs g, T *y) {
  const int64_t grp = blockIdx.x * 256LL + threadIdx.x;
  if (grp >= g.ngroups) return;
  const int64_t b = g.ptr[grp], e = g.ptr[grp + 1];
  for (int c = 0; c < g.ncomp; ++c) {
    T *yc = y + c * g.n_local;
    T s = T(0);
    for (int64_t q = b; q < e; ++q) s += yc[g.idx[q]];
    for (int64_t q = b; q < e; ++q) yc[g.idx[q]] = s;
  }
}

}  // namespace

template <typename T>
hipError_t launch_fill(T *p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_fill<T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interface_sum(const GroupArgs &g, T *y, hipStream_t s) {
  if (g.ngroups == 0) return hipSuccess;
  const int64_t blocks = (g.ngroups + 255) / 256;
  hipLaunchKernelGGL((k_interface<T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, g, y);
  return hipGetLastError();
}

template hipError_t launch_fill<double>(double *, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float *, int64_t, float, hipStream_t);
template hipError_t launch_interface_sum<double>(const GroupArgs &, double *, hipStream_t);
template hipError_t launch_interface_sum<float>(const GroupArgs &, float *, hipStream_t);

}  // namespace tmf
