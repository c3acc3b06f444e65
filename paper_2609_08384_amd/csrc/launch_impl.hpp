// Definitions of the launchers declared in launch.hpp (included only by the
// per-length translation units len_*.hip, which instantiate them).
#pragma once

#include "launch.hpp"

namespace brahms {
namespace detail {

// ---------------------------------------------------------------------------
// plans: each supported axis length maps to a (N1, N2) split with N2 threads
// per line and N1 values per thread
// ---------------------------------------------------------------------------
template <int N1, int N2, int AX, int NF, int NL, int BLOCK = kBlock>
void launch_pass(bool full, dim3 grid, hipStream_t st, const PassArgs& a) {
  if (full) hipLaunchKernelGGL((axis_pass<N1, N2, AX, NF, NL, true, BLOCK>), grid, dim3(BLOCK), 0, st, a);
  else hipLaunchKernelGGL((axis_pass<N1, N2, AX, NF, NL, false, BLOCK>), grid, dim3(BLOCK), 0, st, a);
}

// A linear pass (one field per block) over `lines` lines along AX, with
// kBlock or (wide, where the split has a wide form) kWideBlock threads per
// block.
template <int N1, int N2, int AX>
void launch_linear(bool wide, long lines, int nf, hipStream_t st, const PassArgs& a) {
  if constexpr (wide_split<N1>()) {
    if (wide) {
      constexpr int LPB = LineGeom<N1, N2, kWideBlock>::LPB;
      const dim3 grid(unsigned((lines + LPB - 1) / LPB), 1, unsigned(nf));
      launch_pass<N1, N2, AX, 1, NL_NONE, kWideBlock>(lines % LPB == 0, grid, st, a);
      return;
    }
  }
  constexpr int LPB = LineGeom<N1, N2>::LPB;
  const dim3 grid(unsigned((lines + LPB - 1) / LPB), 1, unsigned(nf));
  launch_pass<N1, N2, AX, 1, NL_NONE>(lines % LPB == 0, grid, st, a);
}

template <int N1, int N2, int AX, int NF>
void launch_nl_nf(int nl, bool full, dim3 grid, hipStream_t st, const PassArgs& a) {
  if constexpr (!long_tau_kind(AX)) {
    if (nl == (NL_AFTER | NL_FUSE)) {
      launch_pass<N1, N2, AX, NF, NL_AFTER | NL_FUSE>(full, grid, st, a);
      return;
    }
  }
  switch (nl) {
    case NL_BEFORE: launch_pass<N1, N2, AX, NF, NL_BEFORE>(full, grid, st, a); break;
    case NL_AFTER: launch_pass<N1, N2, AX, NF, NL_AFTER>(full, grid, st, a); break;
    case NL_BEFORE | NL_MAP: launch_pass<N1, N2, AX, NF, NL_BEFORE | NL_MAP>(full, grid, st, a); break;
    default: launch_pass<N1, N2, AX, NF, NL_AFTER | NL_MAP>(full, grid, st, a); break;
  }
}

template <int N1, int N2, int AX>
void launch_nl(int nf, int nl, bool full, dim3 grid, hipStream_t st, const PassArgs& a) {
  if (nf == 3) launch_nl_nf<N1, N2, AX, 3>(nl, full, grid, st, a);
  else launch_nl_nf<N1, N2, AX, 2>(nl, full, grid, st, a);
}

// Half-step modes without the transverse map: y passes that carry a
// half-step (nt = 1) and the single tau pass of a plane wave (NL_BOTH).
template <int N1, int N2, int AX, int NF>
void launch_plain_nl_nf(int nl, bool full, dim3 grid, hipStream_t st, const PassArgs& a) {
  switch (nl) {
    case NL_BEFORE: launch_pass<N1, N2, AX, NF, NL_BEFORE>(full, grid, st, a); break;
    case NL_AFTER: launch_pass<N1, N2, AX, NF, NL_AFTER>(full, grid, st, a); break;
    case NL_AFTER | NL_FUSE: launch_pass<N1, N2, AX, NF, NL_AFTER | NL_FUSE>(full, grid, st, a); break;
    default: launch_pass<N1, N2, AX, NF, NL_BOTH>(full, grid, st, a); break;
  }
}

template <int N1, int N2, int AX>
void launch_plain_nl(int nf, int nl, bool full, dim3 grid, hipStream_t st, const PassArgs& a) {
  if (nf == 3) launch_plain_nl_nf<N1, N2, AX, 3>(nl, full, grid, st, a);
  else launch_plain_nl_nf<N1, N2, AX, 2>(nl, full, grid, st, a);
}

template <int N1, int N2>
hipError_t launch_axis(int axis, int nl, int nf, const brahms_plan_s& p, PassArgs a) {
  using G = LineGeom<N1, N2>;
  a.tile_mul = 1;
  a.tiles = 1;
  const bool wide = wide_split<N1>() && ((p.wide >> axis) & 1) != 0;
  if (axis == AX_X) {
    const long lines = long(p.ny) * p.nt;
    if (nl == NL_NONE) {
      launch_linear<N1, N2, AX_X>(wide, lines, nf, p.stream, a);
    } else {
      const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB));
      launch_nl<N1, N2, AX_X>(nf, nl, lines % G::LPB == 0, grid, p.stream, a);
    }
  } else if (axis == AX_Y) {
    const long lines = long(p.nx) * p.nt;
    if (nl == NL_NONE) {
      launch_linear<N1, N2, AX_Y>(wide, lines, nf, p.stream, a);
    } else {
      const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB));
      launch_plain_nl<N1, N2, AX_Y>(nf, nl, lines % G::LPB == 0, grid, p.stream, a);
    }
  } else {
    const long lines = long(p.nx) * p.ny;
    const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB));
    a.tile_mul = tile_multiplier(grid.x);
    a.tiles = grid.x;
    if (nl == NL_NONE) {
      // linear tau pass (orders 2 and 3): one field per block, its tiles
      // those of its own block size
      if (wide) {
        constexpr int LPB = LineGeom<N1, N2, kWideBlock>::LPB;
        a.tiles = unsigned((lines + LPB - 1) / LPB);
        a.tile_mul = tile_multiplier(a.tiles);
      }
      launch_linear<N1, N2, AX_T>(wide, lines, nf, p.stream, a);
    } else if (nl == NL_BOTH) {
      launch_plain_nl<N1, N2, AX_T>(nf, nl, lines % G::LPB == 0, grid, p.stream, a);
    } else {
      launch_nl<N1, N2, AX_T>(nf, nl, lines % G::LPB == 0, grid, p.stream, a);
    }
  }
  return hipGetLastError();
}

template <int N1, int N2, int AX>
hipError_t launch_long(int nl, int nf, const brahms_plan_s& p, PassArgs a) {
  using G = LineGeom<N1, N2>;
  a.tile_mul = 1;
  a.tiles = 1;
  const long lines = long(p.nx) * p.ny * (p.nt / G::N);
  const bool full = lines % G::LPB == 0;
  if (AX == AX_TAI && nl != NL_NONE) {
    const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB));
    launch_nl<N1, N2, AX_TAI>(nf, nl, full, grid, p.stream, a);
  } else {
    // linear passes (the inverse b pass too, when fused step pairs carry
    // the RK4 step on x and y): one field per block
    const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB), 1, unsigned(nf));
    launch_pass<N1, N2, AX, 1, NL_NONE>(full, grid, p.stream, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batches: the problem index is a grid dimension (blockIdx.y for passes over
// all fields, blockIdx.z / nf for passes of one field per block)
// ---------------------------------------------------------------------------
template <int N1, int N2, int AX, int NF, int NL, int BLOCK = kBlock>
void launch_batched(bool full, dim3 grid, hipStream_t st, const PassArgs* d, long long step, int nf) {
  if (full)
    hipLaunchKernelGGL((axis_pass_batched<N1, N2, AX, NF, NL, true, BLOCK>), grid, dim3(BLOCK), 0, st, d, step,
                       nf);
  else
    hipLaunchKernelGGL((axis_pass_batched<N1, N2, AX, NF, NL, false, BLOCK>), grid, dim3(BLOCK), 0, st, d, step,
                       nf);
}

// A linear x or y pass over a launch group with kWideBlock threads per block.
template <int N1, int N2, int AX>
void launch_batched_wide(long lines, const GroupGeom& g, hipStream_t st, const PassArgs* d, long long step) {
  if constexpr (wide_split<N1>()) {
    constexpr int LPB = LineGeom<N1, N2, kWideBlock>::LPB;
    const dim3 grid(unsigned((lines + LPB - 1) / LPB), 1, unsigned(g.nf) * g.m);
    launch_batched<N1, N2, AX, 1, NL_NONE, kWideBlock>(lines % LPB == 0, grid, st, d, step, g.nf);
  }
}

template <int N1, int N2, int AX, int NF>
void launch_batched_nl_nf(int nl, bool full, dim3 grid, hipStream_t st, const PassArgs* d, long long step) {
  if constexpr (!long_tau_kind(AX)) {
    if (nl == (NL_AFTER | NL_FUSE)) {
      launch_batched<N1, N2, AX, NF, NL_AFTER | NL_FUSE>(full, grid, st, d, step, NF);
      return;
    }
  }
  switch (nl) {
    case NL_BEFORE: launch_batched<N1, N2, AX, NF, NL_BEFORE>(full, grid, st, d, step, NF); break;
    case NL_AFTER: launch_batched<N1, N2, AX, NF, NL_AFTER>(full, grid, st, d, step, NF); break;
    default: launch_batched<N1, N2, AX, NF, NL_BOTH>(full, grid, st, d, step, NF); break;
  }
}

template <int N1, int N2, int AX>
void launch_batched_nl(int nf, int nl, bool full, dim3 grid, hipStream_t st, const PassArgs* d,
                       long long step) {
  if (nf == 3) launch_batched_nl_nf<N1, N2, AX, 3>(nl, full, grid, st, d, step);
  else launch_batched_nl_nf<N1, N2, AX, 2>(nl, full, grid, st, d, step);
}

template <int N1, int N2>
void launch_group_pass(int axis, int nl, const GroupGeom& g, hipStream_t st, const PassArgs* d,
                       long long step) {
  using G = LineGeom<N1, N2>;
  const unsigned m = g.m;
  const long lines = axis == AX_X ? long(g.ny) * g.nt : (axis == AX_Y ? long(g.nx) * g.nt : long(g.nx) * g.ny);
  const bool full = lines % G::LPB == 0;
  const unsigned blocks = unsigned((lines + G::LPB - 1) / G::LPB);
  if (nl == NL_NONE && axis != AX_T && wide_split<N1>() && ((g.wide >> axis) & 1)) {
    if (axis == AX_X) launch_batched_wide<N1, N2, AX_X>(lines, g, st, d, step);
    else launch_batched_wide<N1, N2, AX_Y>(lines, g, st, d, step);
  } else if (nl == NL_NONE) {
    const dim3 grid(blocks, 1, unsigned(g.nf) * m);
    if (axis == AX_X) launch_batched<N1, N2, AX_X, 1, NL_NONE>(full, grid, st, d, step, g.nf);
    else if (axis == AX_Y) launch_batched<N1, N2, AX_Y, 1, NL_NONE>(full, grid, st, d, step, g.nf);
    else launch_batched<N1, N2, AX_T, 1, NL_NONE>(full, grid, st, d, step, g.nf);
  } else {
    const dim3 grid(blocks, m);
    if (axis == AX_X) launch_batched_nl<N1, N2, AX_X>(g.nf, nl, full, grid, st, d, step);
    else if (axis == AX_Y) launch_batched_nl<N1, N2, AX_Y>(g.nf, nl, full, grid, st, d, step);
    else launch_batched_nl<N1, N2, AX_T>(g.nf, nl, full, grid, st, d, step);
  }
}

template <int N1, int N2, int AX>
void launch_group_long(int nl, const GroupGeom& g, hipStream_t st, const PassArgs* d, long long step) {
  using G = LineGeom<N1, N2>;
  const long lines = long(g.nx) * g.ny * (g.nt / G::N);
  const bool full = lines % G::LPB == 0;
  if constexpr (AX == AX_TAI) {
    const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB), g.m);
    launch_batched_nl<N1, N2, AX_TAI>(g.nf, nl, full, grid, st, d, step);
  } else {
    const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB), 1, unsigned(g.nf) * g.m);
    launch_batched<N1, N2, AX, 1, NL_NONE>(full, grid, st, d, step, g.nf);
  }
}

// ---------------------------------------------------------------------------
// adjoint passes (x or tau, with the VJP of the half-step they undo)
// ---------------------------------------------------------------------------
template <int N1, int N2, int AX, int NF, int AT>
void launch_adj(const brahms_plan_s& p, const AdjArgs& a) {
  using G = LineGeom<N1, N2>;
  const long lines = AX == AX_X ? long(p.ny) * p.nt : long(p.nx) * p.ny;
  const dim3 grid(unsigned((lines + G::LPB - 1) / G::LPB));
  AdjArgs b = a;
  b.tile_mul = AX == AX_T ? tile_multiplier(grid.x) : 1u;
  if (lines % G::LPB == 0)
    hipLaunchKernelGGL((adjoint_pass<N1, N2, AX, NF, AT, true>), grid, dim3(kBlock), 0, p.stream, b);
  else
    hipLaunchKernelGGL((adjoint_pass<N1, N2, AX, NF, AT, false>), grid, dim3(kBlock), 0, p.stream, b);
}

template <int N1, int N2>
void launch_adj_axis(int axis, int at, const brahms_plan_s& p, const AdjArgs& a) {
  if (axis == AX_X) {
    if (p.nf == 3) {
      if (at == VJP_FIRST) launch_adj<N1, N2, AX_X, 3, VJP_FIRST>(p, a);
      else launch_adj<N1, N2, AX_X, 3, VJP_LAST>(p, a);
    } else {
      if (at == VJP_FIRST) launch_adj<N1, N2, AX_X, 2, VJP_FIRST>(p, a);
      else launch_adj<N1, N2, AX_X, 2, VJP_LAST>(p, a);
    }
  } else {
    if (p.nf == 3) {
      if (at == VJP_FIRST) launch_adj<N1, N2, AX_T, 3, VJP_FIRST>(p, a);
      else launch_adj<N1, N2, AX_T, 3, VJP_LAST>(p, a);
    } else {
      if (at == VJP_FIRST) launch_adj<N1, N2, AX_T, 2, VJP_FIRST>(p, a);
      else launch_adj<N1, N2, AX_T, 2, VJP_LAST>(p, a);
    }
  }
}

}  // namespace detail
}  // namespace brahms

// Explicit instantiations of the launchers of one line length.
#define BRAHMS_INSTANTIATE_LENGTH(N1, N2)                                                              \
  template hipError_t brahms::detail::launch_axis<N1, N2>(int, int, int, const brahms_plan_s&,        \
                                                          brahms::PassArgs);                           \
  template void brahms::detail::launch_group_pass<N1, N2>(int, int, const brahms::detail::GroupGeom&, \
                                                          hipStream_t, const brahms::PassArgs*,        \
                                                          long long);                                  \
  template void brahms::detail::launch_adj_axis<N1, N2>(int, int, const brahms_plan_s&,               \
                                                        const brahms::AdjArgs&);

// Explicit instantiations of the three long-tau passes of one sub-length.
#define BRAHMS_INSTANTIATE_LONG_AX(N1, N2, AX)                                                          \
  template hipError_t brahms::detail::launch_long<N1, N2, AX>(int, int, const brahms_plan_s&,          \
                                                              brahms::PassArgs);                        \
  template void brahms::detail::launch_group_long<N1, N2, AX>(int, const brahms::detail::GroupGeom&,   \
                                                              hipStream_t, const brahms::PassArgs*,     \
                                                              long long);
#define BRAHMS_INSTANTIATE_LONG(N, N1, N2)            \
  BRAHMS_INSTANTIATE_LONG_AX(N1, N2, brahms::AX_TAF) \
  BRAHMS_INSTANTIATE_LONG_AX(N1, N2, brahms::AX_TB)  \
  BRAHMS_INSTANTIATE_LONG_AX(N1, N2, brahms::AX_TAI)
