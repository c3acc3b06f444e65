// Axis lengths of the line transforms and their register/lane splits.
//
// A line of length N = N1 N2 is transformed by N2 lanes holding N1 values
// each (see line_fft in kernels.hpp): an N1-point register DFT per lane, one
// exchange through LDS, N2-point register DFTs.  N2 divides N1 (the second
// stage deals N1 / N2 groups to every lane) and kBlock = 256 (a block holds
// 256 / N2 lines), so N2 is a power of two and every factor 3 of N sits in
// N1; N1 and N2 divide 144 (the angles of the register DFTs' constant
// twiddles).  These conditions admit every length 2^a 3^b <= 256 with
// b <= 2: 3^2 N2 lengths take N1 = 9, 18 or 36.  A factor 3^3 would need
// N1 >= 27 values of every field in every lane with N2 = 1, or 54 with N2 =
// 2, beyond the registers of a lane for three fields; those lengths (27, 54,
// 81, 108, 162, 216, 243), other primes, and x or y axes above 256 have no
// split (BRAHMS_E_UNSUPPORTED).  A tau axis of 512, 1024, 2048 or 4096 takes
// three passes of sub-lengths 16, 32 or 64 (a four-step transform, AX_TAF /
// AX_TB / AX_TAI in kernels.hpp).
#pragma once

// X(N, N1, N2) for every supported length of one line transform.
#define BRAHMS_LENGTHS(X)                                                                     \
  X(1, 1, 1) X(2, 2, 1) X(3, 3, 1) X(4, 4, 1) X(6, 6, 1) X(8, 4, 2) X(12, 6, 2) X(16, 4, 4)  \
  X(24, 12, 2) X(32, 8, 4) X(48, 12, 4) X(64, 8, 8) X(96, 24, 4) X(128, 16, 8) X(192, 24, 8) \
  X(256, 16, 16) X(9, 9, 1) X(18, 18, 1) X(36, 18, 2) X(72, 36, 2) X(144, 36, 4)

// X(N, N1, N2): a second split of some lengths, with twice as many lines per
// block (N2 halved) or a whole line per lane.  Which split runs faster depends
// on the grid (lines per launch against values per lane); a plan's schedule
// field `split` picks it per axis and the autotuner times both.
#define BRAHMS_ALT_LENGTHS(X) \
  X(8, 8, 1) X(12, 12, 1) X(16, 8, 2) X(24, 24, 1) X(32, 16, 2) X(48, 24, 2) X(64, 16, 4)

// X(N, N1, N2) for the sub-transform lengths of a long tau axis.
#define BRAHMS_LONG_SUBLENGTHS(X) X(16, 4, 4) X(32, 8, 4) X(64, 8, 8)

namespace brahms {

// Whether n is the length of one line transform.
inline bool line_length(int n) {
#define BRAHMS_CASE_(N, N1, N2) \
  if (n == N) return true;
  BRAHMS_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
  return false;
}

// Whether length n has a second split.
inline bool has_alt_split(int n) {
#define BRAHMS_CASE_(N, N1, N2) \
  if (n == N) return true;
  BRAHMS_ALT_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
  return false;
}

// Lines per block of the transform of length n (256 / N2) with its first
// split, or with its second one when alt is set and it has one; 0 for an
// unsupported length.
inline int lines_per_block(int n, bool alt = false) {
#define BRAHMS_CASE_(N, N1, N2) \
  if (alt && n == N) return 256 / N2;
  BRAHMS_ALT_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
#define BRAHMS_CASE_(N, N1, N2) \
  if (n == N) return 256 / N2;
  BRAHMS_LENGTHS(BRAHMS_CASE_)
#undef BRAHMS_CASE_
  return 0;
}

}  // namespace brahms
