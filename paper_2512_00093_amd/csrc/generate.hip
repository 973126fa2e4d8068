// Bulk generation over many independent streams: one stream per half-wave,
// two per wave64, eight (or, in the wide-store kernel, sixteen) per workgroup
// (see gen_dev.hpp for the mapping).
#include <algorithm>

#include "common.hpp"
#include "gen_dev.hpp"
#include "internal.hpp"

namespace ranmar {

// The stream of half-wave j (0..H-1) of workgroup b in the wide-store kernel
// (H half-waves per workgroup).  The dispatcher hands workgroup b to XCD
// b mod 8, so workgroup 8k + x takes streams 8 (kH + j) + x: neighbouring rows
// of the output are written from different XCDs.  On 2^20 rows of 4 KB this
// measured 4% faster than H neighbouring rows per workgroup (10% without a
// residency cap, and 14% with 16 half-waves per workgroup); on 65,536 rows of
// 16 KB the plain kernel measured 9% slower with it, and keeps eight
// neighbouring rows per workgroup.  Grids are a multiple of 8 workgroups;
// streams past n leave.
template <int H>
__device__ __forceinline__ uint64_t spread_stream(uint32_t b, uint32_t j) {
  return ((uint64_t)(b >> 3) * H + j) * 8u + (b & 7u);
}

template <int FMT, bool NT>
__global__ __launch_bounds__(256) void k_gen32(const uint32_t* __restrict__ sin, uint32_t* sout, uint64_t n,
                                               uint64_t count, void* __restrict__ out, uint64_t ld, uint64_t plane) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t l = lane & 31u;
  const uint64_t s = (uint64_t)blockIdx.x * 8u + (threadIdx.x >> 5);
  if (s >= n) return;  // a whole half-wave leaves together; shifts stay inside a half
  const uint32_t* W = sin + s * kWords;
  char* row = (char*)out + s * ld * 4u;
  if constexpr (FMT == RANMAR_U24_F32) {
    // Both formats as two sweeps over the stream from the same start state
    // (uint32 row, then float row), so that a half-wave has one row in
    // flight at a time, as with one format.
    const StreamRegs st = load_stream(W, l);
    gen_regs32<RANMAR_U24, NT>(l, lane, st, W, nullptr, count, false, row);
    gen_regs32<RANMAR_F32, NT>(l, lane, st, W, sout ? sout + s * kWords : nullptr, count, true, row + plane * 4u);
  } else {
    gen_stream32<FMT, NT>(l, lane, W, sout ? sout + s * kWords : nullptr, count, FMT == RANMAR_F32, row, plane);
  }
}

// Several streams per half-wave: half-wave h takes streams h, h + H, h + 2H,
// ... (H half-waves in the grid) and loads the next stream's state while it
// generates the current one, so short streams do not wait for their state.
template <int FMT, bool NT>
__global__ __launch_bounds__(256) void k_gen32_pipe(const uint32_t* __restrict__ sin, uint32_t* sout, uint64_t n,
                                                    uint64_t count, void* __restrict__ out, uint64_t ld, uint64_t H,
                                                    uint64_t plane) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t l = lane & 31u;
  const uint64_t h = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 2u + (lane >> 5);
  if (h >= n) return;  // a whole half-wave leaves together
  StreamRegs cur = load_stream(sin + h * kWords, l);
  for (uint64_t s = h; s < n; s += H) {
    const uint64_t sn = s + H;
    StreamRegs nxt = cur;
    if (sn < n) nxt = load_stream(sin + sn * kWords, l);  // in flight during the draws below
    gen_regs32<FMT, NT>(l, lane, cur, sin + s * kWords, sout ? sout + s * kWords : nullptr, count,
                        FMT == RANMAR_F32, (char*)out + s * ld * 4u, plane);
    cur = nxt;
  }
}

// Wide-store variant: H half-waves per workgroup (8 or 16), each with a
// 512-byte LDS transpose buffer.
template <int FMT, bool NT, int H>
__global__ __launch_bounds__(32 * H) void k_gen32_wide(const uint32_t* __restrict__ sin, uint32_t* sout, uint64_t n,
                                                       uint64_t count, void* __restrict__ out, uint64_t ld) {
  __shared__ uint32_t bufs[H * 128];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t l = lane & 31u;
  const uint64_t s = spread_stream<H>(blockIdx.x, threadIdx.x >> 5);
  if (s >= n) return;
  gen_stream32_wide<FMT, NT>(l, lane, sin + s * kWords, sout ? sout + s * kWords : nullptr, count,
                             FMT == RANMAR_F32, (char*)out + s * ld * 4u, bufs + (threadIdx.x >> 5) * 128);
}

const char* gen_variant_name(int v) {
  switch (v) {
    case GEN_LANES32: return "lanes32";
    case GEN_LANES32_NT: return "lanes32_nt";
    case GEN_WIDE4: return "lanes32_wide4";
    case GEN_WIDE4_NT: return "lanes32_wide4_nt";
    case GEN_PIPE_NT: return "lanes32_pipe_nt";
    case GEN_LANES32_NT_R2: return "lanes32_nt_res2";
    case GEN_LANES32_NT_R3: return "lanes32_nt_res3";
    case GEN_WIDE4_NT_R4: return "lanes32_wide4_nt_res4";
    case GEN_WIDE4_NT_R6: return "lanes32_wide4_nt_res6";
    case GEN_WIDE4_NT_R5: return "lanes32_wide4_nt_res5";
    case GEN_WIDE16_NT_R2: return "lanes32_wide4_nt_wg16_res2";
    case GEN_WIDE16_NT_R3: return "lanes32_wide4_nt_wg16_res3";
    default: return "?";
  }
}

// Dynamic LDS (unused by the kernel) that leaves room for at most k resident
// workgroups of static LDS `stat` per CU: the smallest per-workgroup total
// above per_cu / (k + 1).  0 (no cap) if the device does not report its LDS.
static unsigned residency_lds(int k, unsigned stat) {
  int dev = 0, per_cu = 0, per_wg = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      hipDeviceGetAttribute(&per_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || per_cu <= 0)
    return 0;
  const unsigned total = ((unsigned)per_cu / (unsigned)(k + 1) + 256u) & ~255u;
  if (total > (unsigned)per_wg || total <= stat) return 0;
  return total - stat;
}

template <int FMT>
static hipError_t launch_fmt(int variant, const uint32_t* sin, uint32_t* sout, uint64_t n, uint64_t count, void* out,
                             uint64_t ld, hipStream_t st) {
  const unsigned wg = 256;
  const uint64_t per_wg = wg / 32;
  const dim3 grid((unsigned)(((n + per_wg - 1) / per_wg + 7) & ~7ull));  // whole groups of 8 (spread_stream)
  const dim3 grid16((unsigned)(((n + 15) / 16 + 7) & ~7ull));             // 16 half-waves per workgroup
  // The wide stores need 16-byte aligned rows, and write one format.
  const bool wide_ok = (((uintptr_t)out & 15) == 0) && (ld % 4 == 0) && FMT != RANMAR_U24_F32;
  const uint64_t plane = n * ld;  // second plane of RANMAR_U24_F32
  unsigned cap_lds = 0;  // residency cap of the _R variants
  if (variant == GEN_LANES32_NT_R2 || variant == GEN_LANES32_NT_R3) {
    cap_lds = residency_lds(variant == GEN_LANES32_NT_R2 ? 2 : 3, 0);
    variant = GEN_LANES32_NT;
  } else if (variant == GEN_WIDE4_NT_R4 || variant == GEN_WIDE4_NT_R5 || variant == GEN_WIDE4_NT_R6) {
    cap_lds = residency_lds(variant == GEN_WIDE4_NT_R4 ? 4 : variant == GEN_WIDE4_NT_R5 ? 5 : 6,
                            wide_ok ? 8 * 128 * 4 : 0);
    variant = GEN_WIDE4_NT;
  } else if (variant == GEN_WIDE16_NT_R2 || variant == GEN_WIDE16_NT_R3) {
    if (wide_ok) {
      cap_lds = residency_lds(variant == GEN_WIDE16_NT_R2 ? 2 : 3, 16 * 128 * 4);
      if constexpr (FMT != RANMAR_U24_F32)
        hipLaunchKernelGGL((k_gen32_wide<FMT, true, 16>), grid16, dim3(512), cap_lds, st, sin, sout, n, count, out,
                           ld);
      return hipGetLastError();
    }
    variant = GEN_LANES32_NT;  // unaligned rows: 4-byte stores
  }
  if (!wide_ok && variant == GEN_WIDE4) variant = GEN_LANES32;
  if (!wide_ok && variant == GEN_WIDE4_NT) variant = GEN_LANES32_NT;
  if (variant == GEN_PIPE_NT) {
    // Enough half-waves for about four times what the device holds at once;
    // each then takes about n / H streams.
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_gen32_pipe<FMT, true>, wg, 0) !=
            hipSuccess || per_cu <= 0)
      per_cu = 8;
    const uint64_t cap = (uint64_t)(cus > 0 ? cus : 256) * (uint64_t)per_cu * per_wg;  // resident half-waves
    uint64_t H = std::min<uint64_t>(n, 4 * cap);
    const dim3 g((unsigned)((H + per_wg - 1) / per_wg));
    H = (uint64_t)g.x * per_wg;  // every half-wave of the grid takes part in the stride
    hipLaunchKernelGGL((k_gen32_pipe<FMT, true>), g, dim3(wg), 0, st, sin, sout, n, count, out, ld, H, plane);
    return hipGetLastError();
  }
  switch (variant) {
    case GEN_WIDE4:
      if constexpr (FMT != RANMAR_U24_F32)
        hipLaunchKernelGGL((k_gen32_wide<FMT, false, 8>), grid, dim3(wg), 0, st, sin, sout, n, count, out, ld);
      break;
    case GEN_WIDE4_NT:
      if constexpr (FMT != RANMAR_U24_F32)
        hipLaunchKernelGGL((k_gen32_wide<FMT, true, 8>), grid, dim3(wg), cap_lds, st, sin, sout, n, count, out, ld);
      break;
    case GEN_LANES32_NT:
      hipLaunchKernelGGL((k_gen32<FMT, true>), grid, dim3(wg), cap_lds, st, sin, sout, n, count, out, ld, plane);
      break;
    default:
      hipLaunchKernelGGL((k_gen32<FMT, false>), grid, dim3(wg), 0, st, sin, sout, n, count, out, ld, plane);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_generate(int variant, const uint32_t* sin, uint32_t* sout, uint64_t n, uint64_t count, int fmt,
                           void* out, uint64_t ld, hipStream_t st) {
  if (!n) return hipSuccess;
  if (fmt == RANMAR_F32) return launch_fmt<RANMAR_F32>(variant, sin, sout, n, count, out, ld, st);
  if (fmt == RANMAR_U24_F32) return launch_fmt<RANMAR_U24_F32>(variant, sin, sout, n, count, out, ld, st);
  return launch_fmt<RANMAR_U24>(variant, sin, sout, n, count, out, ld, st);
}

}  // namespace ranmar
