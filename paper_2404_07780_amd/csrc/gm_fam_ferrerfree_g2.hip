// gm_fam_ferrerfree_g2.hip -- kernels of the model family single Ferrer with free a, b + sky (9 LM variables), 2 plane groups; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_ferrerfree_2() { return make_variant<FamFerrerFree, 2, 15, 25>(); }
}  // namespace gm
