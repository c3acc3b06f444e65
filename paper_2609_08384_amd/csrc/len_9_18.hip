// Pass launchers of plans, batches and the adjoint for line lengths
// 9x1 18x1 18x2 (N1 x N2; see launch.hpp and lengths.hpp).
#include "launch_impl.hpp"

BRAHMS_INSTANTIATE_LENGTH(9, 1)
BRAHMS_INSTANTIATE_LENGTH(18, 1)
BRAHMS_INSTANTIATE_LENGTH(18, 2)
