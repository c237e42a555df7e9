// Issue-rate probe of the vector ALU (measurement support for the roofline
// accounting; declared in rbe_probe.h). Every mix runs on registers only:
// independent chains, so that the SIMD always has an instruction to issue,
// and a final store that keeps every chain alive.
#include "../../include/rbe_probe.h"
#include "kernels.h"

namespace rbe {
namespace {

constexpr int kProbeThreads = 256;

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) k_probe_valu(float *__restrict__ out, int iters, float b, float c,
                                                               unsigned off, unsigned lo) {
  float a[8];
  for (int k = 0; k < 8; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f + 1.0f;
  float px = 0.f, py = 0.f, pz = 0.f;
  const float xi = a[0] * 0.5f, yi = a[1] * 0.25f, zi = a[2] * 0.125f;
  for (int it = 0; it < iters; ++it) {
    if (KIND == RBE_PROBE_FMA_F32 || KIND == RBE_PROBE_RCP_F32 || KIND == RBE_PROBE_MUL_ADD) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          if (KIND == RBE_PROBE_FMA_F32) a[k] = fmaf(a[k], b, c);
          if (KIND == RBE_PROBE_RCP_F32) a[k] = __builtin_amdgcn_rcpf(a[k]);
          // separate multiply and add (the library is built without
          // contraction), the first chain's sum feeding the next's product
          if (KIND == RBE_PROBE_MUL_ADD) a[k] = a[k] + a[(k + 1) & 7] * c;
        }
      }
    } else {
      // four candidates of the LJ tile loop, their coordinates taken from
      // the chains and the results fed back so that no round is dead code
      auto cand = [&](float vx, float vy, float vz) {
        const float dx = xi - vx, dy = yi - vy, dz = zi - vz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const bool in = __float_as_uint(r2) + off >= lo;
        const float ri = __builtin_amdgcn_rcpf(r2);
        const float u3 = ri * ri * ri;
        float f = u3 * fmaf(u3, c, -1.0f) * ri;
        f = in ? f : 0.f;
        px = fmaf(f, dx, px);
        py = fmaf(f, dy, py);
        pz = fmaf(f, dz, pz);
      };
      cand(a[0], a[1], a[2]);
      cand(a[3], a[4], a[5]);
      cand(a[6], a[7], a[0] + b);
      cand(a[1], a[5], a[6]);
      a[0] = fmaf(px, 1e-30f, a[0]);
      a[3] = fmaf(py, 1e-30f, a[3]);
      a[6] = fmaf(pz, 1e-30f, a[6]);
    }
  }
  float s = px + py + pz;
  for (int k = 0; k < 8; ++k) s += a[k];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace rbe

extern "C" int rbe_probe_valu(int kind, int blocks, int iters, float *out, float *ms, void *stream) {
  using namespace rbe;
  if (kind < RBE_PROBE_FMA_F32 || kind > RBE_PROBE_RCP_F32) return fail_without_context(RBE_EINVAL, "unknown probe kind");
  if (blocks < 1 || iters < 1) return fail_without_context(RBE_EINVAL, "blocks and iters must be at least 1");
  if (!out || !ms) return fail_without_context(RBE_EINVAL, "out or ms is NULL");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail_without_context(RBE_EDEVICE, "hipEventCreate failed");
  }
  // r^2 + off >= lo as in the tile loop (off = ~bits(lo_r2), lo = -bits(lo_r2))
  const unsigned lo_bits = __builtin_bit_cast(unsigned, 6.25f);
  const float b = 1.0000001f, c = 1e-7f;
  const unsigned off = ~lo_bits, lo = 0u - lo_bits;
  (void)hipEventRecord(e0, st);
  switch (kind) {
    case RBE_PROBE_FMA_F32:
      k_probe_valu<RBE_PROBE_FMA_F32><<<blocks, kProbeThreads, 0, st>>>(out, iters, b, c, off, lo);
      break;
    case RBE_PROBE_MUL_ADD:
      k_probe_valu<RBE_PROBE_MUL_ADD><<<blocks, kProbeThreads, 0, st>>>(out, iters, b, c, off, lo);
      break;
    case RBE_PROBE_LJ_BODY:
      k_probe_valu<RBE_PROBE_LJ_BODY><<<blocks, kProbeThreads, 0, st>>>(out, iters, b, c, off, lo);
      break;
    default:
      k_probe_valu<RBE_PROBE_RCP_F32><<<blocks, kProbeThreads, 0, st>>>(out, iters, b, c, off, lo);
      break;
  }
  (void)hipEventRecord(e1, st);
  const hipError_t err = hipGetLastError() != hipSuccess ? hipErrorLaunchFailure : hipEventSynchronize(e1);
  float t = 0.f;
  const bool ok = err == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return fail_without_context(RBE_EDEVICE, "probe launch or its events failed");
  *ms = t;
  return RBE_OK;
}
