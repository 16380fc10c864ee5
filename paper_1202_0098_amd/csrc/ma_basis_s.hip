// On-chip basis kernel k_basis_s instantiated for o = 4 and any o, 256 or
// 512 threads, subspace capacity 16 or 32, and every precision mode.
#include "ma_device.h"

namespace ma {

namespace {

template <int O, int NT, int NU>
void *pick(int prec)
{
    if (prec == 1) return (void *)k_basis_s<O, NT, NU, 1>;
    if (prec == 2) return (void *)k_basis_s<O, NT, NU, 2>;
    return (void *)k_basis_s<O, NT, NU, 0>;
}

}  // namespace

void *basis_s_kernel(int o, int nt, int nucap, int prec)
{
    if (o == 4) {
        if (nt == 256) return nucap == 16 ? pick<4, 256, 16>(prec) : pick<4, 256, 32>(prec);
        return nucap == 16 ? pick<4, 512, 16>(prec) : pick<4, 512, 32>(prec);
    }
    if (nt == 256) return nucap == 16 ? pick<0, 256, 16>(prec) : pick<0, 256, 32>(prec);
    return nucap == 16 ? pick<0, 512, 16>(prec) : pick<0, 512, 32>(prec);
}

}  // namespace ma
