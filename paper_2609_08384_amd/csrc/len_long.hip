// Launchers of the three passes of a long tau axis (sub-transforms of 16, 32
// and 64 points; see launch.hpp and lengths.hpp).
#include "launch_impl.hpp"

BRAHMS_LONG_SUBLENGTHS(BRAHMS_INSTANTIATE_LONG)
