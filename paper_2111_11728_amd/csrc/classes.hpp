// Classes of subdomain-local DOFs shared by the host topology and the kernels.
#pragma once

#include <cstdint>

namespace feti {

// interior (i), interface touched by constraint rows (b), FETI-DP corner (c), clamped (x)
enum : int8_t { CLS_I = 0, CLS_B = 1, CLS_C = 2, CLS_X = 3 };

}  // namespace feti
