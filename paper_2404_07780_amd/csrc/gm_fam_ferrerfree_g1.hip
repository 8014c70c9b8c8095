// gm_fam_ferrerfree_g1.hip -- kernels of the model family single Ferrer with free a, b + sky (9 LM variables), 1 plane group; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_ferrerfree_1() { return make_variant<FamFerrerFree, 1, 15, 25>(); }
}  // namespace gm
