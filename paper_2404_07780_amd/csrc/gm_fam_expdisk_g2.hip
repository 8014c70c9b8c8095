// gm_fam_expdisk_g2.hip -- kernels of the model family exponential disk + sky, 2 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_expdisk_2() { return make_variant<FamSingle<ExpDisk>, 2, 25>(); }
}  // namespace gm
