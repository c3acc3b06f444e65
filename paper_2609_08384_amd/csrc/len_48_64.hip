// Pass launchers of plans, batches and the adjoint for line lengths
// 12x4 8x8 (N1 x N2; see launch.hpp and lengths.hpp), and second splits.
#include "launch_impl.hpp"

BRAHMS_INSTANTIATE_LENGTH(12, 4)
BRAHMS_INSTANTIATE_LENGTH(8, 8)
// second splits (lengths.hpp: BRAHMS_ALT_LENGTHS)
BRAHMS_INSTANTIATE_LENGTH(24, 2)
BRAHMS_INSTANTIATE_LENGTH(16, 4)
