// gm_fam_moffat.hip -- kernels of the model family: Moffat + sky (7).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_moffat() { return make_ops<FamSingle<Moffat>, 2, 25>(); }
}  // namespace gm
