// Workspace basis kernel k_basis_g instantiated for o = 9 (0: any o) and
// every rows-per-thread count and precision mode.
#include "ma_device.h"

namespace ma {

namespace {

template <int R>
void *pick(int prec)
{
    if (prec == 1) return (void *)k_basis_g<9, R, 1>;
    if (prec == 2) return (void *)k_basis_g<9, R, 2>;
    return (void *)k_basis_g<9, R, 0>;
}

}  // namespace

void *basis_g_kernel_o9(int R, int prec)
{
    switch (R) {
    case 1: return pick<1>(prec);
    case 2: return pick<2>(prec);
    case 3: return pick<3>(prec);
    case 4: return pick<4>(prec);
    case 6: return pick<6>(prec);
    default: return pick<8>(prec);
    }
}

}  // namespace ma
