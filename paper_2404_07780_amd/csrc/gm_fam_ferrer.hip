// gm_fam_ferrer.hip -- kernels of the model family: Ferrer + sky (7).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_ferrer() { return make_ops<FamSingle<Ferrer>, 2, 25>(); }
}  // namespace gm
