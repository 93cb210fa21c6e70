// Learned edgeMap-variant selector (placeholder until the MLP lands).
#include "internal.h"

namespace byo {

int mlp_choose_variant(const level_features &f, bool allow_pull) {
  (void)f;
  (void)allow_pull;
  return -1;
}

}  // namespace byo
