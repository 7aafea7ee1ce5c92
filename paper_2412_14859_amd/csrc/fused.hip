// Single-pass fused step (not yet available: the two-pass path is used).
#include "internal.hpp"

namespace cge {

bool fused_supported(const cge_ctx*) { return false; }
long long fused_blocks(const cge_ctx*) { return 0; }
cge_status fused_steps(cge_ctx* c, long long) {
    return fail(c, CGE_EUNSUPPORTED, "fused step kernel not available");
}

}  // namespace cge
