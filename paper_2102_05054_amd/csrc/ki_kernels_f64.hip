// complex128 instances of the kicked-Ising kernels.
#include "ki_kernels_impl.h"

namespace fq {

template hipError_t ki_launch_pass<double>(const KiPassArgs<double>&, int, int, bool, unsigned, hipStream_t,
                                           unsigned);
template hipError_t ki_launch_pass3<double>(const KiPassArgs<double>&, int, unsigned, hipStream_t, unsigned);
template hipError_t ki_launch_pipe<double>(const KiPassArgs<double>&, int, int, bool, unsigned, unsigned, unsigned,
                                          hipStream_t);
template hipError_t ki_launch_single<double>(const KiSingleArgs<double>&, int, int, bool, bool, unsigned,
                                             hipStream_t, bool);

}  // namespace fq
