// Bandwidth probes for CDNA4 (gfx950): the ceilings the remap and section
// kernels are measured against.
//
// stream_*: plain 16-byte streams over a buffer -- read only, write only,
// and copy (read + write, the access pattern of a remap) -- with a
// persistent grid, every wave issuing coalesced 1 KiB accesses; the host
// takes the best of a sweep of forms (1, 2, 4 or 8 chunks in flight per
// thread, ordinary or streaming accesses, 4, 8 or 16 workgroups per CU, the
// grid striding over the buffer or each workgroup streaming a contiguous
// share of it).
// gather: random accesses of 4, 8 or 16 bytes at record r * stride for
// uniformly random records r (the access of a gather section's neighbour
// field), one per lane, the index array and the per-lane results streamed.
// Its time per access, together with the HBM bytes the counters report,
// gives the bytes one random access really fetches (the access granule).
#include <algorithm>
#include <vector>

#include "adha_impl.h"

namespace adha {

typedef uint32_t u32x4p __attribute__((ext_vector_type(4)));

// U: 16-byte chunks per thread per step, all loaded before any is used;
// NT: streaming (non-temporal) accesses.  Thread t of workgroup w handles
// chunks (i * G + w) * 256 * U + t + 256 * u, so each wave access is 1 KiB
// of consecutive bytes.
template <bool NT>
__device__ __forceinline__ u32x4p ld16(const u32x4p *p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st16(u32x4p *p, u32x4p v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// The chunks a thread visits: from `first`, steps of `step` below `end`.
// Grid-striding (CONT = false): workgroup w starts at w * 256 * U and the
// grid moves over the buffer together.  Contiguous (CONT = true): workgroup
// w streams chunks [w * share, (w + 1) * share), share a multiple of 256 * U.
template <int U, bool CONT>
__device__ __forceinline__ void chunk_range(uint64_t n16, uint64_t *first, uint64_t *end, uint64_t *step) {
  if constexpr (CONT) {
    const uint64_t per = 256ull * U;
    const uint64_t share = (n16 + (uint64_t)gridDim.x * per - 1) / ((uint64_t)gridDim.x * per) * per;
    *first = (uint64_t)blockIdx.x * share + threadIdx.x;
    *end = std::min<uint64_t>(n16, (uint64_t)(blockIdx.x + 1) * share);
    *step = per;
  } else {
    *first = (uint64_t)blockIdx.x * 256 * U + threadIdx.x;
    *end = n16;
    *step = (uint64_t)gridDim.x * 256 * U;
  }
}

template <int U, bool NT, bool CONT>
__global__ __launch_bounds__(256) void probe_read_kernel(const u32x4p *__restrict__ a, uint64_t n16,
                                                         uint32_t *__restrict__ sink) {
  u32x4p acc = {0, 0, 0, 0};
  uint64_t i, end, step;
  chunk_range<U, CONT>(n16, &i, &end, &step);
  for (; i < end; i += step) {
    u32x4p v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = i + 256 * u < end ? ld16<NT>(a + i + 256 * u) : u32x4p{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u];
  }
  // one word per thread, written only when the xor is a value no buffer of
  // the probe holds, so the store traffic stays out of the measurement
  const uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
  if (x == 0x9E3779B9u) sink[(uint64_t)blockIdx.x * 256 + threadIdx.x] = x;
}

template <int U, bool NT, bool CONT>
__global__ __launch_bounds__(256) void probe_write_kernel(u32x4p *__restrict__ b, uint64_t n16, uint32_t v) {
  const u32x4p w = {v, v ^ 1u, v ^ 2u, v ^ 3u};
  uint64_t i, end, step;
  chunk_range<U, CONT>(n16, &i, &end, &step);
  for (; i < end; i += step) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + 256 * u < end) st16<NT>(b + i + 256 * u, w);
  }
}

template <int U, bool NT, bool CONT>
__global__ __launch_bounds__(256) void probe_copy_kernel(const u32x4p *__restrict__ a, u32x4p *__restrict__ b,
                                                         uint64_t n16) {
  uint64_t i, end, step;
  chunk_range<U, CONT>(n16, &i, &end, &step);
  for (; i < end; i += step) {
    u32x4p v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + 256 * u < end) v[u] = ld16<NT>(a + i + 256 * u);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + 256 * u < end) st16<NT>(b + i + 256 * u, v[u]);
  }
}

// LB bytes from the start of record idx[i]: one load of 4 or 8 bytes, or
// LB / 16 loads of 16 bytes (up to a whole 128-byte line).
template <int LB>
__global__ __launch_bounds__(256) void probe_gather_kernel(const uint8_t *__restrict__ buf, uint64_t stride,
                                                           const int32_t *__restrict__ idx, uint64_t n,
                                                           uint32_t *__restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint8_t *p = buf + (uint64_t)(uint32_t)idx[i] * stride;
    uint32_t v;
    if constexpr (LB == 4) {
      v = *reinterpret_cast<const uint32_t *>(p);
    } else if constexpr (LB == 8) {
      const uint2 q = *reinterpret_cast<const uint2 *>(p);
      v = q.x ^ q.y;
    } else {
      u32x4p q[LB / 16];
#pragma unroll
      for (int u = 0; u < LB / 16; ++u) q[u] = reinterpret_cast<const u32x4p *>(p)[u];
      u32x4p acc = q[0];
#pragma unroll
      for (int u = 1; u < LB / 16; ++u) acc ^= q[u];
      v = acc.x ^ acc.y ^ acc.z ^ acc.w;
    }
    out[i] = v;
  }
}

}  // namespace adha

using namespace adha;

namespace {

template <class Fn>
adha_status median_us(hipStream_t st, uint32_t reps, Fn fn, double *out) {
  hipEvent_t a, b;
  ADHA_HIP(hipEventCreate(&a));
  ADHA_HIP(hipEventCreate(&b));
  std::vector<double> ts;
  hipError_t e = hipSuccess;
  fn();
  for (uint32_t r = 0; r < std::max(1u, reps) && e == hipSuccess; ++r) {
    (void)hipEventRecord(a, st);
    fn();
    (void)hipEventRecord(b, st);
    e = hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    ts.push_back(ms * 1e3);
  }
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(ADHA_ERR_DEVICE, "probe failed: %s", hipGetErrorString(e));
  std::sort(ts.begin(), ts.end());
  *out = ts[ts.size() / 2];
  return ADHA_OK;
}

}  // namespace

extern "C" {

adha_status adha_probe_stream(adha_ctx *ctx, uint32_t kind, void *a, void *b, uint64_t bytes, uint32_t reps,
                              void *stream, double *us) {
  if (!ctx || !us) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (kind > 2) return fail(ADHA_ERR_INVALID, "kind %u is not 0 (read), 1 (write) or 2 (copy)", kind);
  if (bytes == 0 || bytes % 16) return fail(ADHA_ERR_INVALID, "bytes must be a positive multiple of 16");
  if (((uintptr_t)a & 255u) || ((uintptr_t)b & 255u)) return fail(ADHA_ERR_INVALID, "buffers must be 256-byte aligned");
  if ((kind != 1 && !a) || !b) return fail(ADHA_ERR_INVALID, "a buffer is NULL");
  const uint64_t n16 = bytes / 16;
  if (kind == 2 && (uintptr_t)a < (uintptr_t)b + bytes && (uintptr_t)b < (uintptr_t)a + bytes)
    return fail(ADHA_ERR_INVALID, "source and destination overlap");
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  // the best of the sweep: U chunks in flight per thread (1, 2, 4, 8),
  // ordinary or streaming accesses, 4, 8 or 16 workgroups per CU, grid-
  // striding or contiguous shares
  double best = 0.0;
  bool have = false;
  for (uint32_t wpc : {4u, 8u, 16u})
    for (int U : {1, 2, 4, 8})
      for (int nt = 0; nt < 2; ++nt)
        for (int cont = 0; cont < 2; ++cont) {
          const uint32_t grid = (uint32_t)std::max<uint64_t>(
              1, std::min<uint64_t>((n16 + 256 * U - 1) / (256 * U), (uint64_t)ctx->c.cu_count * wpc));
          // the read probe's sink holds one word per thread of the grid
          if (kind == 0 && (uint64_t)grid * 256 * 4 > bytes) continue;
          double t = 0.0;
#define ADHA_PROBE(UU, NTT, CC)                                                                                  \
  ADHA_TRY(median_us(st, reps, [&] {                                                                             \
    if (kind == 0)                                                                                               \
      hipLaunchKernelGGL((probe_read_kernel<UU, NTT, CC>), dim3(grid), dim3(256), 0, st, (const u32x4p *)a, n16, \
                         (uint32_t *)b);                                                                         \
    else if (kind == 1)                                                                                          \
      hipLaunchKernelGGL((probe_write_kernel<UU, NTT, CC>), dim3(grid), dim3(256), 0, st, (u32x4p *)b, n16,      \
                         0x5A5A5A5Au);                                                                           \
    else                                                                                                         \
      hipLaunchKernelGGL((probe_copy_kernel<UU, NTT, CC>), dim3(grid), dim3(256), 0, st, (const u32x4p *)a,      \
                         (u32x4p *)b, n16);                                                                      \
  }, &t))
#define ADHA_PROBE_U(UU)                                \
  if (nt && cont) ADHA_PROBE(UU, true, true);           \
  else if (nt) ADHA_PROBE(UU, true, false);             \
  else if (cont) ADHA_PROBE(UU, false, true);           \
  else ADHA_PROBE(UU, false, false);
          if (U == 1) { ADHA_PROBE_U(1) }
          else if (U == 2) { ADHA_PROBE_U(2) }
          else if (U == 4) { ADHA_PROBE_U(4) }
          else { ADHA_PROBE_U(8) }
#undef ADHA_PROBE_U
#undef ADHA_PROBE
          if (!have || t < best) best = t;
          have = true;
        }
  if (!have) return fail(ADHA_ERR_INVALID, "buffer too small for the probe");
  *us = best;
  return ADHA_OK;
}

adha_status adha_probe_gather(adha_ctx *ctx, const void *buf, uint64_t buf_bytes, uint64_t stride,
                              uint32_t load_bytes, const int32_t *idx, uint64_t n, void *out, uint32_t reps,
                              void *stream, double *us) {
  if (!ctx || !us || !buf || !idx || !out) return fail(ADHA_ERR_INVALID, "NULL argument");
  if (load_bytes != 4 && load_bytes != 8 && load_bytes != 16 && load_bytes != 32 && load_bytes != 64 &&
      load_bytes != 128)
    return fail(ADHA_ERR_INVALID, "load_bytes is 4, 8, 16, 32, 64 or 128");
  if (stride < load_bytes || stride % load_bytes) return fail(ADHA_ERR_INVALID, "stride must be a multiple of load_bytes");
  if (((uintptr_t)buf & 255u) || ((uintptr_t)idx & 255u) || ((uintptr_t)out & 255u))
    return fail(ADHA_ERR_INVALID, "buffers must be 256-byte aligned");
  if (n == 0 || n > (1ull << 28)) return fail(ADHA_ERR_INVALID, "n must be in [1, 2^28]");
  // every index must name a record inside buf: records = buf_bytes / stride;
  // the caller's indices are checked on the host before any launch
  const uint64_t records = buf_bytes / stride;
  if (records == 0 || records > (1ull << 31)) return fail(ADHA_ERR_INVALID, "buf holds %llu records",
                                                          (unsigned long long)records);
  std::vector<int32_t> h(n);
  DeviceGuard g(ctx->c.device);
  hipStream_t st = (hipStream_t)stream;
  ADHA_HIP(hipMemcpyAsync(h.data(), idx, n * 4, hipMemcpyDeviceToHost, st));
  ADHA_HIP(hipStreamSynchronize(st));
  for (uint64_t i = 0; i < n; ++i)
    if (h[i] < 0 || (uint64_t)h[i] >= records)
      return fail(ADHA_ERR_INVALID, "index %llu = %d is outside [0, %llu)", (unsigned long long)i, h[i],
                  (unsigned long long)records);
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, (uint64_t)ctx->c.cu_count * 16);
  const uint8_t *p = (const uint8_t *)buf;
  return median_us(st, reps, [&] {
#define ADHA_GATHER(LB) \
  hipLaunchKernelGGL(probe_gather_kernel<LB>, dim3(grid), dim3(256), 0, st, p, stride, idx, n, (uint32_t *)out)
    switch (load_bytes) {
      case 4: ADHA_GATHER(4); break;
      case 8: ADHA_GATHER(8); break;
      case 16: ADHA_GATHER(16); break;
      case 32: ADHA_GATHER(32); break;
      case 64: ADHA_GATHER(64); break;
      default: ADHA_GATHER(128); break;
    }
#undef ADHA_GATHER
  }, us);
}

}  // extern "C"
