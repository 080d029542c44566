// Boundary-MPS contraction, norms, energies and two-site updates (internals).
#pragma once
#include "esvd.h"

namespace hp {}  // namespace hp
