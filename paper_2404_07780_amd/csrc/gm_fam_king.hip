// gm_fam_king.hip -- kernels of the model family: King + sky (8).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_king() { return make_ops<FamSingle<King>, 2, 25>(); }
}  // namespace gm
