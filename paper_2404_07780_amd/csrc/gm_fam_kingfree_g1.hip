// gm_fam_kingfree_g1.hip -- kernels of the model family single King with free alpha + sky (9 LM variables), 1 plane group; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_kingfree_1() { return make_variant<FamKingFree, 1, 15, 25>(); }
}  // namespace gm
