// Standalone map launches (plain scheduler and captured graph chains): the
// partition pass, then the merge pass, over the jobs registered by the last
// epoch.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "map.h"

namespace trees {

// Map launches (plain and graph forms).  from_hdr: take the job count the
// last scan recorded; the merge launch clears it when done so that a later
// launch in a captured chain does not repeat it.
template <int WG, int TILE>
__global__ __launch_bounds__(WG) void k_map_part(DevCtx C, uint32_t Jarg, int32_t from_hdr) {
  const uint32_t Jraw = from_hdr ? C.hdr->mapJ : Jarg;
  if (!Jraw) return;
  uint32_t J;
  uint64_t U;
  map_extent<TILE>(C, Jraw, &J, &U);
  // Only the work-groups that one boundary per wavefront needs take part
  // (a captured chain launches a grid sized for the largest map).  Work-
  // groups are dispatched round-robin over the 8 XCDs (block b on XCD b % 8);
  // renumbered this way, each XCD searches a contiguous run of boundaries,
  // whose shared upper probes then hit in its own L2, and every XCD gets
  // an equal share.
  const uint64_t nb = (U + TILE - 1) / TILE + 1;
  const uint64_t need = (nb + WG / 64 - 1) / (WG / 64);
  uint32_t G = gridDim.x;
  if (G % 8 == 0 && need < G) G = (uint32_t)((need + 7) & ~(uint64_t)7);
  if (blockIdx.x >= G) return;
  const uint32_t v = (G % 8 == 0) ? (blockIdx.x % 8) * (G / 8) + blockIdx.x / 8 : blockIdx.x;
  map_partition<TILE>(C, J, U, (int64_t)v * (WG / 64) + (threadIdx.x >> 6), (int64_t)G * (WG / 64));
}

// 2048 lanes per CU (8 wavefronts per SIMD): at most 64 registers a lane.
template <int WG, int TILE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(8)))
void k_map_merge(DevCtx C, uint32_t Jarg, int32_t from_hdr) {
  __shared__ MapLds<TILE> M;
  const uint32_t Jraw = from_hdr ? C.hdr->mapJ : Jarg;
  if (!Jraw) return;
  uint32_t J;
  uint64_t U;
  map_extent<TILE>(C, Jraw, &J, &U);
  map_merge<WG, TILE, true>(map_view(C), M, J, U);
  if (from_hdr) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t a = add_agent(&C.hdr->map_arrive, 1u);
      if (a == gridDim.x - 1) {
        st_agent(&C.hdr->map_arrive, 0u);
        st_agent(&C.hdr->mapJ, 0u);
      }
    }
  }
}

// Map launches: the partition pass then the merge pass.  grid_part and
// grid_merge are work-group counts (both passes loop over their work).
// ev (may be null): four HIP events, the start and end of each pass.
hipError_t launch_map(const DevCtx &C, int wg, uint32_t jobs, int from_hdr, int grid_part, int grid_merge,
                      hipStream_t s, const hipEvent_t *ev) {
  const void *fp = nullptr, *fm = nullptr;
  switch (wg) {
    case kMapWG:
      fp = (const void *)&k_map_part<kMapWG, kMapLaunchTile>;
      fm = (const void *)&k_map_merge<kMapWG, kMapLaunchTile>;
      break;
    default: return hipErrorInvalidValue;
  }
  DevCtx c = C;
  uint32_t j = jobs;
  int32_t f = from_hdr;
  void *args[] = {&c, &j, &f};
  hipError_t e = hipExtLaunchKernel(fp, dim3(grid_part), dim3(wg), args, 0, s, ev ? ev[0] : nullptr,
                                    ev ? ev[1] : nullptr, 0);
  if (e != hipSuccess) return e;
  return hipExtLaunchKernel(fm, dim3(grid_merge), dim3(wg), args, 0, s, ev ? ev[2] : nullptr,
                            ev ? ev[3] : nullptr, 0);
}

}  // namespace trees
