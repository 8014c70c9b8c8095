// gm_fam_king_g1.hip -- kernels of the model family King + sky, 1 plane group; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_king_1() { return make_variant<FamSingle<King>, 1, 25>(); }
}  // namespace gm
