// Treecode forward and adjoint (filled in below).
#include "rism_internal.h"

namespace rism {

int tree_forward(const TreeCallArgs &, Workspace &, rism_stats &, hipStream_t)
{
    set_error("RISM_TREECODE: not built yet");
    return RISM_E_UNSUPPORTED;
}

int tree_forward_cp(const TreeCallArgs &, Workspace &, rism_stats &, hipStream_t)
{
    set_error("RISM_TREECODE_CP: not built yet");
    return RISM_E_UNSUPPORTED;
}

int adjoint_tree(const AdjointArgs &, Workspace &, rism_stats &, hipStream_t)
{
    set_error("RISM_TREECODE backward: not built yet");
    return RISM_E_UNSUPPORTED;
}

}  // namespace rism
