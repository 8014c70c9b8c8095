// gm_fam_moffat_g2.hip -- kernels of the model family Moffat + sky, 2 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_moffat_2() { return make_variant<FamSingle<Moffat>, 2, 25>(); }
}  // namespace gm
