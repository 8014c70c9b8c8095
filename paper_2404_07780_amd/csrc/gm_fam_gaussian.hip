// gm_fam_gaussian.hip -- kernels of the model family: Gaussian + sky (7).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_gaussian() { return make_ops<FamSingle<Gaussian>, 2, 25>(); }
}  // namespace gm
