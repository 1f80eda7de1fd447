// Hex kernel instantiations for order p = 1, n_q = p+1 .. p+3 and 9 (9^3 points).
#include "kernels3d.hpp"
#include "ops.hpp"
#include "tiles3.hpp"

namespace tmop {

bool ops3_p1(int nq, Ops *out)
{
    switch (nq) {
    case 1 + 1: TMOP_OPS_BODY(k3, S3, 1, 1 + 1)
    case 1 + 2: TMOP_OPS_BODY(k3, S3, 1, 1 + 2)
    case 1 + 3: TMOP_OPS_BODY(k3, S3, 1, 1 + 3)
    case 9: TMOP_OPS_BODY(k3, S3, 1, 9)
    default: return false;
    }
}

bool bops3_p1(int nq, BOps *out)
{
    switch (nq) {
    case 1 + 1: TMOP_BOPS_BODY(kb3, S3, 1, 1 + 1)
    case 1 + 2: TMOP_BOPS_BODY(kb3, S3, 1, 1 + 2)
    case 1 + 3: TMOP_BOPS_BODY(kb3, S3, 1, 1 + 3)
    case 9: TMOP_BOPS_BODY(kb3, S3, 1, 9)
    default: return false;
    }
}

}  // namespace tmop
