// Four-step pass kernels and launchers instantiated for double.
#include "fourstep.hpp"

namespace amg {

template hipError_t launch_col_fwd<double>(int, const LevelDev<double>&, const ColIn<double>&, cplx<double>*,
                                       const Twiddles<double>&, double*, hipStream_t);
template hipError_t launch_row<double>(int, const LevelDev<double>&, cplx<double>*, const Twiddles<double>&,
                                   const double*, int, const double*, hipStream_t);
template hipError_t launch_col_inv<double>(int, const LevelDev<double>&, const EpiOut<double>&,
                                       const cplx<double>*, const Twiddles<double>&, double*, hipStream_t);

template hipError_t launch_col_fwd_batch<double>(int, const LevelDev<double>&, const PassArgs<double>*, int,
                                                 const Twiddles<double>&, hipStream_t);
template hipError_t launch_row_batch<double>(const LevelDev<double>&, const PassArgs<double>*, int,
                                         const Twiddles<double>&, hipStream_t);
template hipError_t launch_col_inv_batch<double>(int, const LevelDev<double>&, const PassArgs<double>*, int,
                                             const Twiddles<double>&, hipStream_t);

}  // namespace amg
