// Instantiations of the HALS / MU local-update kernels for k = 1..44.
#include "local_kernels.h"

void nmf::local::fill_k1_44(LaunchFn* t) { fill<1>(t, std::make_integer_sequence<int, 44>{}); }
