// Instantiations of the HALS / MU local-update kernels for k = 45..56.
#include "local_kernels.h"

void nmf::local::fill_k45_56(LaunchFn* t) { fill<45>(t, std::make_integer_sequence<int, 12>{}); }
