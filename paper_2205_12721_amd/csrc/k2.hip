// Quad kernel instantiations for p = 1..4, n_q = p+1 .. p+3.
#include "kernels2d.hpp"
#include "ops.hpp"

namespace tmop {

bool ops2(int p, int nq, Ops *out)
{
#define TMOP_CASE(P, NQ) \
    if (p == P && nq == NQ) TMOP_OPS_BODY(k2, S2, P, NQ)
    TMOP_CASE(1, 2) TMOP_CASE(1, 3) TMOP_CASE(1, 4)
    TMOP_CASE(2, 3) TMOP_CASE(2, 4) TMOP_CASE(2, 5)
    TMOP_CASE(3, 4) TMOP_CASE(3, 5) TMOP_CASE(3, 6)
    TMOP_CASE(4, 5) TMOP_CASE(4, 6) TMOP_CASE(4, 7)
#undef TMOP_CASE
    return false;
}

bool bops2(int p, int nq, BOps *out)
{
#define TMOP_CASE(P, NQ) \
    if (p == P && nq == NQ) TMOP_BOPS_BODY(kb2, S2, P, NQ)
    TMOP_CASE(1, 2) TMOP_CASE(1, 3) TMOP_CASE(1, 4)
    TMOP_CASE(2, 3) TMOP_CASE(2, 4) TMOP_CASE(2, 5)
    TMOP_CASE(3, 4) TMOP_CASE(3, 5) TMOP_CASE(3, 6)
    TMOP_CASE(4, 5) TMOP_CASE(4, 6) TMOP_CASE(4, 7)
#undef TMOP_CASE
    return false;
}

bool find_bops(int dim, int p, int nq, BOps *out)
{
    if (dim == 2) return bops2(p, nq, out);
    if (dim != 3) return false;
    switch (p) {
    case 1: return bops3_p1(nq, out);
    case 2: return bops3_p2(nq, out);
    case 3: return bops3_p3(nq, out);
    case 4: return bops3_p4(nq, out);
    default: return false;
    }
}

bool find_ops(int dim, int p, int nq, Ops *out)
{
    if (dim == 2) return ops2(p, nq, out);
    if (dim != 3) return false;
    switch (p) {
    case 1: return ops3_p1(nq, out);
    case 2: return ops3_p2(nq, out);
    case 3: return ops3_p3(nq, out);
    case 4: return ops3_p4(nq, out);
    default: return false;
    }
}

}  // namespace tmop
