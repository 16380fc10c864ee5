// Atom-group basis kernel k_basis_m: 512 threads; sp3 (o = 4) regions up to
// 512 orbitals with the 4 columns of an atom together, spd (o = 9) regions up
// to 1,024 orbitals (two rows per thread) with 3 columns together.
#include "ma_device.h"

namespace ma {

namespace {

template <int O, int B, int R>
void *pick(int prec)
{
    if (prec == 1) return (void *)k_basis_m<O, B, 512, R, 1>;
    if (prec == 2) return (void *)k_basis_m<O, B, 512, R, 2>;
    return (void *)k_basis_m<O, B, 512, R, 0>;
}

}  // namespace

void *basis_m_kernel(int o, int prec)
{
    return o == 9 ? pick<9, 3, 2>(prec) : pick<4, 4, 1>(prec);
}

}  // namespace ma
