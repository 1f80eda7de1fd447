// Hex kernel instantiations for order p = 4, n_q = p+1 .. p+3 and 9 (9^3 points).
#include "kernels3d.hpp"
#include "ops.hpp"
#include "tiles3.hpp"

namespace tmop {

bool ops3_p4(int nq, Ops *out)
{
    switch (nq) {
    case 4 + 1: TMOP_OPS_BODY(k3, S3, 4, 4 + 1)
    case 4 + 2: TMOP_OPS_BODY(k3, S3, 4, 4 + 2)
    case 4 + 3: TMOP_OPS_BODY(k3, S3, 4, 4 + 3)
    case 9: TMOP_OPS_BODY(k3, S3, 4, 9)
    default: return false;
    }
}

bool bops3_p4(int nq, BOps *out)
{
    switch (nq) {
    case 4 + 1: TMOP_BOPS_BODY(kb3, S3, 4, 4 + 1)
    case 4 + 2: TMOP_BOPS_BODY(kb3, S3, 4, 4 + 2)
    case 4 + 3: TMOP_BOPS_BODY(kb3, S3, 4, 4 + 3)
    case 9: TMOP_BOPS_BODY(kb3, S3, 4, 9)
    default: return false;
    }
}

}  // namespace tmop
