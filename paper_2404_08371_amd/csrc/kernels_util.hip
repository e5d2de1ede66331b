// Small kernels: fills and the interface sum over duplicated DoFs.
#include "tmf_internal.h"

namespace tmf {

namespace {

// 16-byte stores over the 16-byte-aligned body, scalar stores for the ends
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *p, int64_t n, T v) {
  constexpr int W = 16 / sizeof(T);
  const int64_t head = ((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / sizeof(T);
  const int64_t h = head < n ? head : n;
  const int64_t nv = (n - h) / W;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  const int64_t tid = blockIdx.x * 256LL + threadIdx.x;
  typedef T V __attribute__((ext_vector_type(W)));
  V vv;
  for (int q = 0; q < W; ++q) vv[q] = v;
  V *pv = reinterpret_cast<V *>(p + h);
  for (int64_t i = tid; i < nv; i += stride) pv[i] = vv;
  if (tid < h) p[tid] = v;
  const int64_t tail = h + nv * W;
  if (tid < n - tail) p[tail + tid] = v;
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
  int64_t blocks = (n / (16 / sizeof(T)) + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
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
