// gm_fam_kingfree_g2.hip -- kernels of the model family single King with free alpha + sky (9 LM variables), 2 plane groups; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_kingfree_2() { return make_variant<FamKingFree, 2, 15, 25>(); }
}  // namespace gm
