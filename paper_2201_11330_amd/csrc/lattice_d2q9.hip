// D2Q9 instantiation of the liblbm.so kernels.
#include "impl.hpp"

namespace imexlbm {

const Ops* ops_d2q9(lbm_storage s) { return make_ops<0>(s); }

}  // namespace imexlbm
