// Native worklist BFS and SSSP for CDNA4 (gfx950): the hand-managed
// formulation that Section 6.3 compares TREES with.
//
// Each iteration is one kernel over an input worklist of vertices.  A vertex
// relaxes its out-arcs: BFS claims an unreached head by compare-and-swap of
// its depth (-1 -> level + 1), SSSP lowers the head's distance by an atomic
// min.  A head that is claimed or improved is pushed to the output worklist,
// whose single tail counter is advanced atomically.  After the kernel the
// host reads that one count back; the lists swap and the next kernel covers
// the old output list, until an iteration pushes nothing.
//
// On this chip the worklist kernel uses the same work-group co-operation as
// the TREES epoch kernel, so the two are compared on equal footing: a
// work-group takes 1024 worklist entries, scans their out-degrees in LDS and
// spreads the arcs over its lanes; pushed vertices are staged in LDS and
// reserved in the output list with one device atomic per work-group flush.
// The count reaches the host through host-mapped memory, written by the
// iteration's last work-group (a ticket counter), which the host polls.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "prims.h"
#include "trees_dev.h"

namespace trees {

constexpr int kWlQueue = 2048;   // pushed vertices staged in LDS before a flush

template <int WG>
constexpr int wl_arcs_per_lane() {
  return (kWlQueue / 2) / WG >= 4 ? 4 : ((kWlQueue / 2) / WG > 0 ? (kWlQueue / 2) / WG : 1);
}

template <int WG, bool SSSP>
__global__ __launch_bounds__(WG) void k_wl(WlArgs A) {
  constexpr int IT = kWlChunk / WG;          // worklist entries per lane
  constexpr int AR = wl_arcs_per_lane<WG>();  // arcs per lane per expansion step
  static_assert(WG * AR <= kWlQueue / 2, "staging queue too small for one step");
  __shared__ int32_t s_pre[kWlChunk];   // exclusive prefix of out-degrees, lane-major
  __shared__ int32_t s_row[kWlChunk];   // first arc of each entry's vertex
  __shared__ int32_t s_dv[kWlChunk];    // SSSP: the vertex's distance when loaded
  __shared__ int32_t s_q[kWlQueue];
  __shared__ int32_t s_qn;
  __shared__ uint32_t s_qbase;
  __shared__ int32_t s_tmp[WG / 64 + 1];
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && tid == 0) A.ctl->tail[A.par ^ 1] = 0;   // the next iteration's counter
  if (tid == 0) s_qn = 0;
  const uint32_t base = blockIdx.x * (uint32_t)kWlChunk;

  // ---- entries of this work-group: vertex, first arc, out-degree -----------
  int32_t v[IT], deg[IT], rw[IT], dv[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const uint32_t i = base + (uint32_t)(tid * IT + k);
    v[k] = i < A.n_in ? A.in[i] : -1;
  }
  int dsum = 0;
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    deg[k] = 0; rw[k] = 0; dv[k] = 0;
    if (v[k] >= 0) {
      rw[k] = A.row[v[k]];
      deg[k] = A.row[v[k] + 1] - rw[k];
      if (SSSP) dv[k] = ld_agent(&A.val[v[k]]);   // its distance as it stands now
    }
    dsum += deg[k];
  }
  int tot;
  int pre = wg_excl_scan<WG>(dsum, s_tmp, &tot);
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    s_pre[tid * IT + k] = pre;
    s_row[tid * IT + k] = rw[k];
    if (SSSP) s_dv[tid * IT + k] = dv[k];
    pre += deg[k];
  }
  __syncthreads();

  // ---- arcs spread over the lanes ------------------------------------------
  int from = 0;   // arcs go in increasing order: each lane's item search only moves forward
  for (int e0 = 0; e0 < tot; e0 += WG * AR) {
    int32_t u[AR], nd[AR], cur[AR];
    bool ok[AR];
#pragma unroll
    for (int a = 0; a < AR; ++a) {
      const int e = e0 + a * WG + tid;
      ok[a] = e < tot;
      u[a] = 0; nd[a] = 0;
      if (ok[a]) {
        int lo = from, hi = kWlChunk;   // last entry whose prefix is <= e
        while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_pre[mid] <= e) lo = mid; else hi = mid; }
        from = lo;
        const int32_t arc = s_row[lo] + (e - s_pre[lo]);
        u[a] = A.col[arc];
        if (SSSP) nd[a] = s_dv[lo] + A.w[arc];
      }
    }
#pragma unroll
    for (int a = 0; a < AR; ++a) cur[a] = ok[a] ? A.val[u[a]] : 0;   // probes issued together
#pragma unroll
    for (int a = 0; a < AR; ++a) {
      if (!ok[a]) continue;
      bool push = false;
      if (SSSP) {
        // a lower distance: the head is pushed once per iteration at most
        if (nd[a] < cur[a] && atomicMin(&A.val[u[a]], nd[a]) > nd[a])
          push = atomicExch(&A.stamp[u[a]], A.level) != A.level;
      } else {
        push = cur[a] == -1 && atomicCAS(&A.val[u[a]], -1, A.level + 1) == -1;
      }
      if (push) s_q[atomicAdd(&s_qn, 1)] = u[a];
    }
    __syncthreads();
    const int qn = s_qn;
    if (qn > kWlQueue - WG * AR || e0 + WG * AR >= tot) {
      // flush: one reservation in the output list for the whole queue
      if (tid == 0 && qn > 0) s_qbase = add_agent(&A.ctl->tail[A.par], (uint32_t)qn);
      __syncthreads();
      for (int q = tid; q < qn; q += WG) A.out[s_qbase + (uint32_t)q] = s_q[q];
      __syncthreads();
      if (tid == 0) s_qn = 0;
      __syncthreads();
    }
  }

  // ---- the iteration's last work-group publishes the output count ----------
  // (every work-group's tail reservation returned before it takes a ticket)
  __syncthreads();
  if (tid == 0) {
    const uint32_t t = add_agent(&A.ctl->ticket, 1u);
    if (t + 1 == A.nwg) {
      st_agent(&A.ctl->ticket, 0u);
      __hip_atomic_store(&A.mir->count, ld_agent(&A.ctl->tail[A.par]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
      wait_vmem();
      __hip_atomic_store(&A.mir->seq, A.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// Before the first iteration: every value `fill` except the source's (0), no
// vertex pushed yet, the input list {source}, counters cleared.
__global__ void k_wl_init(int32_t *val, int32_t *stamp, int32_t V, int32_t src, int32_t fill, int32_t *in,
                          WlCtl *ctl) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < V; x += step) {
    val[x] = (x == src) ? 0 : fill;
    if (stamp) stamp[x] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    in[0] = src;
    ctl->tail[0] = 0;
    ctl->tail[1] = 0;
    ctl->ticket = 0;
  }
}

hipError_t launch_wl(const WlArgs &a, int wg, bool sssp, hipStream_t s) {
  const void *fn = nullptr;
  switch (wg) {
    case 256: fn = sssp ? (const void *)&k_wl<256, true> : (const void *)&k_wl<256, false>; break;
    case 512: fn = sssp ? (const void *)&k_wl<512, true> : (const void *)&k_wl<512, false>; break;
    case 1024: fn = sssp ? (const void *)&k_wl<1024, true> : (const void *)&k_wl<1024, false>; break;
    default: return hipErrorInvalidValue;
  }
  if (a.n_in == 0) return hipErrorInvalidValue;
  WlArgs p = a;
  p.nwg = (a.n_in + kWlChunk - 1) / kWlChunk;
  void *args[] = {&p};
  return hipLaunchKernel(fn, dim3(p.nwg), dim3(wg), args, 0, s);
}

hipError_t launch_wl_init(int32_t *val, int32_t *stamp, int32_t V, int32_t src, int32_t fill, int32_t *in,
                          void *ctl, hipStream_t s) {
  WlCtl *c = (WlCtl *)ctl;
  void *args[] = {&val, &stamp, &V, &src, &fill, &in, &c};
  int blocks = (int)((V + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  return hipLaunchKernel((const void *)&k_wl_init, dim3(blocks), dim3(256), args, 0, s);
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free worklist BFS: a fixed array in device
// memory (each GPU the library runs on holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address, taken once per device at context creation, is kept below.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kWlScratchBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// With `device` current: record the device address of its scratch array.
hipError_t wl_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

// The device address recorded for `device`, or null before its setup.
void *wl_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}

size_t wl_ctl_bytes() { return sizeof(WlCtl); }
size_t wl_args_size() { return sizeof(WlArgs); }

}  // namespace trees
