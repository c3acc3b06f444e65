// Pass launchers of plans, batches and the adjoint for line lengths
// 36x2 (N1 x N2; see launch.hpp and lengths.hpp).
#include "launch_impl.hpp"

BRAHMS_INSTANTIATE_LENGTH(36, 2)
