// Local generalised eigenproblems of the GenEO coarse space (see below).
#include "precond.h"

namespace geneo {

void solve_local_gevps(geneo_ctx* ctx, geneo_precond* pc) {
  (void)ctx;
  (void)pc;
  throw Error(GENEO_EUNSUPPORTED, "GenEO eigensolver not built yet");
}

}  // namespace geneo
