// Hex kernel instantiations for order p = 3, n_q = p+1 .. p+3 and 9 (9^3 points).
#include "kernels3d.hpp"
#include "ops.hpp"
#include "tiles3.hpp"

namespace tmop {

bool ops3_p3(int nq, Ops *out)
{
    switch (nq) {
    case 3 + 1: TMOP_OPS_BODY(k3, S3, 3, 3 + 1)
    case 3 + 2: TMOP_OPS_BODY(k3, S3, 3, 3 + 2)
    case 3 + 3: TMOP_OPS_BODY(k3, S3, 3, 3 + 3)
    case 9: TMOP_OPS_BODY(k3, S3, 3, 9)
    default: return false;
    }
}

bool bops3_p3(int nq, BOps *out)
{
    switch (nq) {
    case 3 + 1: TMOP_BOPS_BODY(kb3, S3, 3, 3 + 1)
    case 3 + 2: TMOP_BOPS_BODY(kb3, S3, 3, 3 + 2)
    case 3 + 3: TMOP_BOPS_BODY(kb3, S3, 3, 3 + 3)
    case 9: TMOP_BOPS_BODY(kb3, S3, 3, 9)
    default: return false;
    }
}

}  // namespace tmop
