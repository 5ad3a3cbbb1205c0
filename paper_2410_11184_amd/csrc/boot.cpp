// Bootstrapping: placeholder until the CoeffToSlot / EvalMod / SlotToCoeff
// pipeline is configured for the context.
#include "host.h"
#include "softmax.h"

namespace hs {

bool can_bootstrap(const Context& c) { return false && c.prm.boot.cts_levels > 0; }

Ct bootstrap(Context& c, const Ct& x, double bound) {
    (void)x;
    (void)bound;
    HS_REQUIRE(can_bootstrap(c), E_LEVEL, "bootstrapping is not configured for this context");
    return Ct();
}

}  // namespace hs
