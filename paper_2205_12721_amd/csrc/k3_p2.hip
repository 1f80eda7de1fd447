// Hex kernel instantiations for order p = 2, n_q = p+1 .. p+3 and 9 (9^3 points).
#include "kernels3d.hpp"
#include "ops.hpp"
#include "tiles3.hpp"

namespace tmop {

bool ops3_p2(int nq, Ops *out)
{
    switch (nq) {
    case 2 + 1: TMOP_OPS_BODY(k3, S3, 2, 2 + 1)
    case 2 + 2: TMOP_OPS_BODY(k3, S3, 2, 2 + 2)
    case 2 + 3: TMOP_OPS_BODY(k3, S3, 2, 2 + 3)
    case 9: TMOP_OPS_BODY(k3, S3, 2, 9)
    default: return false;
    }
}

bool bops3_p2(int nq, BOps *out)
{
    switch (nq) {
    case 2 + 1: TMOP_BOPS_BODY(kb3, S3, 2, 2 + 1)
    case 2 + 2: TMOP_BOPS_BODY(kb3, S3, 2, 2 + 2)
    case 2 + 3: TMOP_BOPS_BODY(kb3, S3, 2, 2 + 3)
    case 9: TMOP_BOPS_BODY(kb3, S3, 2, 9)
    default: return false;
    }
}

}  // namespace tmop
