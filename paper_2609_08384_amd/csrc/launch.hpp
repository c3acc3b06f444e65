// Launchers of the pass kernels, one set per line-transform length (declared
// here, defined in launch_impl.hpp, instantiated per length in len_*.hip so
// that the lengths compile in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include "adjoint.hpp"
#include "kernels.hpp"
#include "lengths.hpp"
#include "plan.hpp"

namespace brahms {
namespace detail {

// One pass of a plan along `axis` with lines of length N1 N2; nl says where
// the RK4 step goes (NL_* of kernels.hpp); linear passes take one field per
// block.
template <int N1, int N2>
hipError_t launch_axis(int axis, int nl, int nf, const brahms_plan_s& p, PassArgs a);

// One of the three passes of a long tau axis (sub-transforms N1 N2).
template <int N1, int N2, int AX>
hipError_t launch_long(int nl, int nf, const brahms_plan_s& p, PassArgs a);

// Geometry of a batch launch group: m problems of one shape and field count;
// wide: bits (x = 1, y = 2) of the axes whose linear passes run kWideBlock
// threads per block.
struct GroupGeom {
  unsigned m;
  int nx, ny, nt, nf;
  int wide;
};

// One pass over a launch group (descriptors d[m] of this step).
template <int N1, int N2>
void launch_group_pass(int axis, int nl, const GroupGeom& g, hipStream_t st, const PassArgs* d,
                       long long step);

// One of the three passes of a long tau axis over a launch group.
template <int N1, int N2, int AX>
void launch_group_long(int nl, const GroupGeom& g, hipStream_t st, const PassArgs* d, long long step);

// One adjoint pass (conj-propagator transforms with the RK4 half-step's VJP)
// along x or tau (VJP_FIRST / VJP_LAST of adjoint.hpp).
template <int N1, int N2>
void launch_adj_axis(int axis, int at, const brahms_plan_s& p, const AdjArgs& a);

}  // namespace detail
}  // namespace brahms
