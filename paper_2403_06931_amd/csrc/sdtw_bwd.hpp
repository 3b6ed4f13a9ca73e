// sdtw_bwd.hpp -- backward (adjoint) kernels.
#pragma once
#include "sdtw_common.hpp"
