// gm_fam_king_g2.hip -- kernels of the model family King + sky, 2 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_king_2() { return make_variant<FamSingle<King>, 2, 25>(); }
}  // namespace gm
