// Instantiations of the HALS / MU local-update kernels for k = 57..64.
#include "local_kernels.h"

void nmf::local::fill_k57_64(LaunchFn* t) { fill<57>(t, std::make_integer_sequence<int, 8>{}); }
