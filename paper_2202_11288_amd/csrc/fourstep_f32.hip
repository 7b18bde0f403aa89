// Four-step pass kernels and launchers instantiated for float.
#include "fourstep.hpp"

namespace amg {

template hipError_t launch_col_fwd<float>(int, const LevelDev<float>&, const ColIn<float>&, cplx<float>*,
                                       const Twiddles<float>&, float*, hipStream_t);
template hipError_t launch_row<float>(int, const LevelDev<float>&, cplx<float>*, const Twiddles<float>&,
                                   const float*, int, const float*, hipStream_t);
template hipError_t launch_col_inv<float>(int, const LevelDev<float>&, const EpiOut<float>&,
                                       const cplx<float>*, const Twiddles<float>&, double*, hipStream_t);

template hipError_t launch_col_fwd_batch<float>(int, const LevelDev<float>&, const PassArgs<float>*, int,
                                                 const Twiddles<float>&, hipStream_t);
template hipError_t launch_row_batch<float>(const LevelDev<float>&, const PassArgs<float>*, int,
                                         const Twiddles<float>&, hipStream_t);
template hipError_t launch_col_inv_batch<float>(int, const LevelDev<float>&, const PassArgs<float>*, int,
                                             const Twiddles<float>&, hipStream_t);

}  // namespace amg
