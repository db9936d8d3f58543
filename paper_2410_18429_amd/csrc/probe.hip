// Streaming bandwidth probe: the HBM access mixes of the fused CGLS launches
// with none of their arithmetic, so that the fraction of the 8 TB/s peak that
// the fused kernels reach can be set against what a plain streaming kernel
// with the same reads and writes reaches on the same device.  A measurement
// helper of the library, not a step of the method.
//
// Launch shapes: a grid of 8 blocks of 256 threads per compute unit that
// strides over the arrays (one or four element pairs in flight per thread),
// and a full grid with one element pair per thread, whose blocks sweep memory
// in dispatch order; the full grid is the faster one on MI355X (about 6.3
// against 4.8-5.7 TB/s for a copy), so it sets the ceiling.
#include "../../include/wri.h"
#include "wri_impl.hpp"

#include <cstdint>

namespace wri {
namespace {

// Elements are complex64 (8 B) as in the solver's vectors, processed two per
// thread with 16-byte accesses; m is one float32 per element.  Every thread
// issues the loads of U element pairs (a grid stride apart) before its first
// store, so that enough bytes are in flight; outputs use non-temporal (NT = 1)
// or ordinary stores.  The probe reports the best of the variants.
//   mix 0  copy              read a               write c          16 B / element
//   mix 1  forward           read a, b, m         write c          28 B
//   mix 2  forward + x step  read a, b, m, x, q   write c, x       52 B
//   mix 3  adjoint           read a, b, m         write c, d       36 B
typedef float v4f __attribute__((ext_vector_type(4)));
template <int NT>
__device__ __forceinline__ void st4(float4* p, float4 v) {
  if constexpr (NT != 0) {
    const v4f w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<v4f*>(p));
  } else {
    *p = v;
  }
}

template <int MIX, int NT>
__device__ __forceinline__ void mix_store(int64_t i, float4 va, float4 vb, float2 vm, float4 vx, float4 vq,
                                          float4* __restrict__ c, float4* __restrict__ d, float4* __restrict__ x) {
  if constexpr (MIX == 0) {
    st4<NT>(c + i, va);
  } else {
    float4 r;
    r.x = va.x + vm.x * vb.x; r.y = va.y + vm.x * vb.y;
    r.z = va.z + vm.y * vb.z; r.w = va.w + vm.y * vb.w;
    st4<NT>(c + i, r);
    if constexpr (MIX == 2) {
      float4 y;
      y.x = vx.x + vq.x * vm.x; y.y = vx.y + vq.y * vm.x;
      y.z = vx.z + vq.z * vm.y; y.w = vx.w + vq.w * vm.y;
      st4<NT>(x + i, y);
    }
    if constexpr (MIX == 3) {
      float4 t;
      t.x = va.x - vb.x; t.y = va.y - vb.y; t.z = va.z - vb.z; t.w = va.w - vb.w;
      st4<NT>(d + i, t);
    }
  }
}

template <int MIX, int U, int NT>
__global__ void __launch_bounds__(256)
k_stream(const float4* __restrict__ a, const float4* __restrict__ b, const float2* __restrict__ m,
         float4* __restrict__ c, float4* __restrict__ d, float4* __restrict__ x, const float4* __restrict__ q,
         int64_t npairs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (; i + (U - 1) * stride < npairs; i += U * stride) {
    float4 va[U], vb[U], vx[U], vq[U];
    float2 vm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = i + u * stride;
      va[u] = a[k];
      vb[u] = (MIX != 0) ? b[k] : z4;
      vm[u] = (MIX != 0) ? m[k] : make_float2(0.f, 0.f);
      vx[u] = (MIX == 2) ? x[k] : z4;
      vq[u] = (MIX == 2) ? q[k] : z4;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) mix_store<MIX, NT>(i + u * stride, va[u], vb[u], vm[u], vx[u], vq[u], c, d, x);
  }
  for (; i < npairs; i += stride) {
    const float4 va = a[i];
    const float4 vb = (MIX != 0) ? b[i] : z4;
    const float2 vm = (MIX != 0) ? m[i] : make_float2(0.f, 0.f);
    const float4 vx = (MIX == 2) ? x[i] : z4, vq = (MIX == 2) ? q[i] : z4;
    mix_store<MIX, NT>(i, va, vb, vm, vx, vq, c, d, x);
  }
}

constexpr int kMixBytes[4] = {16, 28, 52, 36};
constexpr size_t kSlot = 256;

size_t round_up(size_t v) { return (v + kSlot - 1) / kSlot * kSlot; }

// workspace: arrays a, b, c, d, x, q of n complex64 each, then m (n float32)
size_t probe_bytes(int64_t n) { return 6 * round_up((size_t)n * 8) + round_up((size_t)n * 4) + kSlot; }

// Tile-order probe: block b -> tile b / n_sys of grid b % n_sys (the same
// tile of consecutive grids on adjacent blocks); each thread moves four cells
// of every plane of the 64 x 16 x 32 tile-slab, loads before stores.
constexpr int kPX = 64, kPY = 16, kPZ = 32;
__global__ void __launch_bounds__(256)
k_tile_stream(const float2* __restrict__ a, const float2* __restrict__ b, const float* __restrict__ m,
              float2* __restrict__ c, int nx, int ny, int nz, int n_sys) {
  typedef float v2f __attribute__((ext_vector_type(2)));
  const int sys = blockIdx.x % n_sys, tile = blockIdx.x / n_sys;
  const int tiles_x = nx / kPX, tiles_y = ny / kPY;
  const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
  const int64_t n = (int64_t)nx * ny * nz, base = (int64_t)sys * n;
  int off[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cell = threadIdx.x + q * 256;
    off[q] = (ty * kPY + cell / kPX) * nx + tx * kPX + cell % kPX;
  }
  const int64_t plane = (int64_t)nx * ny;
  for (int z = tz * kPZ; z < (tz + 1) * kPZ; ++z) {
    float2 va[4], vb[4];
    float vm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = z * plane + off[q];
      va[q] = a[base + i];
      vb[q] = b[base + i];
      vm[q] = m[i];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = z * plane + off[q];
      const v2f w = {va[q].x + vm[q] * vb[q].x, va[q].y + vm[q] * vb[q].y};
      __builtin_nontemporal_store(w, reinterpret_cast<v2f*>(c + base + i));
    }
  }
}

size_t tile_probe_bytes(int64_t cells, int n_sys) {
  return 3 * round_up((size_t)cells * n_sys * 8) + round_up((size_t)cells * 4) + kSlot;
}

}  // namespace
}  // namespace wri

using namespace wri;

extern "C" {

size_t wri_stream_probe_bytes(int32_t mix, int64_t n) {
  if (mix < 0 || mix > 3 || n <= 0 || (n & 1)) return 0;
  return probe_bytes(n);
}

int wri_stream_probe(int32_t mix, int64_t n, int32_t reps, void* ws, size_t ws_bytes, void* stream,
                     double* gbs_out) {
  if (mix < 0 || mix > 3) return report_error(WRI_EINVAL, "wri_stream_probe: mix must be 0..3");
  if (n <= 0 || (n & 1)) return report_error(WRI_EINVAL, "wri_stream_probe: n must be even and positive");
  if (reps < 1) return report_error(WRI_EINVAL, "wri_stream_probe: reps must be >= 1");
  if (gbs_out == nullptr) return report_error(WRI_EINVAL, "wri_stream_probe: gbs_out is NULL");
  if (ws == nullptr || ws_bytes < probe_bytes(n))
    return report_error(WRI_ENOWS, "wri_stream_probe: workspace of %zu bytes is smaller than the %zu required",
                        ws_bytes, probe_bytes(n));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + kSlot - 1) / kSlot * kSlot);
  const size_t vb = round_up((size_t)n * 8);
  float4* arr[6];
  for (int i = 0; i < 6; ++i) arr[i] = reinterpret_cast<float4*>(base + i * vb);
  const float2* m = reinterpret_cast<const float2*>(base + 6 * vb);
  const int64_t npairs = n / 2;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return report_error(WRI_EHIP, "wri_stream_probe: hipEventCreate failed");
  double best = 0.0;
  int rc = WRI_OK;
  // variants: U = 1 and 4 element pairs in flight per thread, ordinary and
  // non-temporal stores, on a grid of 8 blocks of 256 threads per compute unit
  // (var 0-3), and U = 1 on the full grid of one pair per thread (var 4, 5)
  for (int var = 0; var < 6 && rc == WRI_OK; ++var) {
    const int u4 = (var < 4) ? (var >> 1) : 0, nt = var & 1;
    const int64_t want = (npairs + 255) / 256;
    const int64_t cap = (var < 4) ? 2048 : 0x7fffffff;
    const unsigned blocks = (unsigned)(want < cap ? want : cap);
    for (int r = 0; r <= reps && rc == WRI_OK; ++r) {  // launch 0 of a variant is a warm-up
      if (hipEventRecord(e0, st) != hipSuccess) { rc = WRI_EHIP; break; }
#define LAUNCH(M, U, NT)                                                                                    \
  hipLaunchKernelGGL((k_stream<M, U, NT>), dim3(blocks), dim3(256), 0, st, arr[0], arr[1], m, arr[2], arr[3], \
                     arr[4], arr[5], npairs)
#define LAUNCH_MIX(M)                                         \
  if (u4 && nt) LAUNCH(M, 4, 1);                              \
  else if (u4) LAUNCH(M, 4, 0);                               \
  else if (nt) LAUNCH(M, 1, 1);                               \
  else LAUNCH(M, 1, 0);
      switch (mix) {
        case 0: LAUNCH_MIX(0); break;
        case 1: LAUNCH_MIX(1); break;
        case 2: LAUNCH_MIX(2); break;
        default: LAUNCH_MIX(3); break;
      }
#undef LAUNCH_MIX
#undef LAUNCH
      if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess) {
        rc = WRI_EHIP;
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = WRI_EHIP; break; }
      if (r > 0 && ms > 0.f) {
        const double gbs = (double)kMixBytes[mix] * (double)n / (ms * 1e-3) / 1e9;
        if (gbs > best) best = gbs;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != WRI_OK) return report_error(rc, "wri_stream_probe: HIP call failed");
  *gbs_out = best;
  return WRI_OK;
}

size_t wri_tile_probe_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t n_sys) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_sys <= 0 || nx % kPX || ny % kPY || nz % kPZ) return 0;
  return tile_probe_bytes((int64_t)nx * ny * nz, n_sys);
}

int wri_tile_probe(int32_t nx, int32_t ny, int32_t nz, int32_t n_sys, int32_t reps, void* ws, size_t ws_bytes,
                   void* stream, double* gbs_out) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_sys <= 0 || nx % kPX || ny % kPY || nz % kPZ)
    return report_error(WRI_EINVAL, "wri_tile_probe: nx, ny, nz must be positive multiples of %d, %d, %d", kPX, kPY,
                        kPZ);
  const int64_t cells = (int64_t)nx * ny * nz;
  if (cells * n_sys > ((int64_t)1 << 31) || cells > ((int64_t)1 << 28))
    return report_error(WRI_EINVAL, "wri_tile_probe: %lld cells in all are too many", (long long)(cells * n_sys));
  if (reps < 1) return report_error(WRI_EINVAL, "wri_tile_probe: reps must be >= 1");
  if (gbs_out == nullptr) return report_error(WRI_EINVAL, "wri_tile_probe: gbs_out is NULL");
  if (ws == nullptr || ws_bytes < tile_probe_bytes(cells, n_sys))
    return report_error(WRI_ENOWS, "wri_tile_probe: workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                        tile_probe_bytes(cells, n_sys));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + kSlot - 1) / kSlot * kSlot);
  const size_t vb = round_up((size_t)cells * n_sys * 8);
  const float2* a = reinterpret_cast<const float2*>(base);
  const float2* b = reinterpret_cast<const float2*>(base + vb);
  float2* c = reinterpret_cast<float2*>(base + 2 * vb);
  const float* m = reinterpret_cast<const float*>(base + 3 * vb);
  const unsigned blocks = (unsigned)(n_sys * (nx / kPX) * (ny / kPY) * (nz / kPZ));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return report_error(WRI_EHIP, "wri_tile_probe: hipEventCreate failed");
  double best = 0.0;
  int rc = WRI_OK;
  for (int r = 0; r <= reps && rc == WRI_OK; ++r) {  // launch 0 is a warm-up
    float ms = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess) { rc = WRI_EHIP; break; }
    hipLaunchKernelGGL(k_tile_stream, dim3(blocks), dim3(256), 0, st, a, b, m, c, nx, ny, nz, n_sys);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = WRI_EHIP;
      break;
    }
    if (r > 0 && ms > 0.f) {
      const double gbs = 28.0 * (double)cells * n_sys / (ms * 1e-3) / 1e9;
      if (gbs > best) best = gbs;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != WRI_OK) return report_error(rc, "wri_tile_probe: HIP call failed");
  *gbs_out = best;
  return WRI_OK;
}

}  // extern "C"
