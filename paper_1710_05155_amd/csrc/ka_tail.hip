// ka_tail.hip -- the trailing run of tiny classes of a general graph in one launch (gfx950).
//
// Method: Boccagna, arXiv 1710.05155; the per-edge bit logic lives in ka_device.h.  A greedy
// distance-2 colouring ends in a few classes of a few hundred edges or fewer; launched one
// by one, each would cost a whole launch's ramp and drain for a few thousand loads.
#include "ka_device.h"

namespace ka {
namespace {

using namespace dev;

// A run of consecutive small classes [a.c, a.c_end) of a general graph in one launch: one
// workgroup per plane runs them in order, with a workgroup barrier between classes.  During
// the launch only this workgroup touches the plane's words, and the barrier orders its
// stores before its later loads (workgroup scope: all its waves run on one CU), so every
// class sees the previous one complete, as across separate launches.  Same-class edges
// commute, so a thread may take several of them in any order.
template <int Z, int WPT>
__global__ __launch_bounds__(kTailEdges) void k_tail_graph(PassGraph a, int m)
{
  const int plane = a.plane0 + (int)blockIdx.x;
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  u64 *n = a.n + off, *f = a.f + off;
  for (uint32_t c = a.c; c < a.c_end; ++c) {
    const int b0 = a.class_start[c], b1 = a.class_start[c + 1];
    for (int k = b0 + (int)threadIdx.x; k < b1; k += kTailEdges) {
      if (a.fsat)
        graph_edge<Z, WPT>(n, f, a.edges, a.nbr, a.stride, k, plane, m, a.t, c, a.key0, a.key1, a.noise,
                           FSat{a.fsat, plane * a.N});
      else
        graph_edge<Z, WPT>(n, f, a.edges, a.nbr, a.stride, k, plane, m, a.t, c, a.key0, a.key1, a.noise);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_tail_graph(const PassGraph &a, int z, int m, int wpt, hipStream_t s)
{
  if (!a.class_start || a.c_end <= a.c || a.planes < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)a.planes), block((unsigned)kTailEdges);
#define KA_TG(Z, W) hipLaunchKernelGGL((k_tail_graph<Z, W>), grid, block, 0, s, a, m)
  switch (z * 4 + wpt) {
    case 3 * 4 + 1: KA_TG(3, 1); break;
    case 3 * 4 + 2: KA_TG(3, 2); break;
    case 4 * 4 + 1: KA_TG(4, 1); break;
    case 4 * 4 + 2: KA_TG(4, 2); break;
    case 5 * 4 + 1: KA_TG(5, 1); break;
    case 5 * 4 + 2: KA_TG(5, 2); break;
    case 6 * 4 + 1: KA_TG(6, 1); break;
    case 6 * 4 + 2: KA_TG(6, 2); break;
    default: return hipErrorInvalidValue;
  }
#undef KA_TG
  return hipGetLastError();
}

}  // namespace ka
