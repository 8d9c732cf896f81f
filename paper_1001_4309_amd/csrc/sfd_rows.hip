// Row pass kernels (the x transforms, see row_body) and their launcher.
#include "sfd_device.h"

namespace sfd {

template <int L, int GR, int VAR, int P>
__global__ void __launch_bounds__((PassShape<L, GR, P>::THREADS)) __attribute__((amdgpu_waves_per_eu(SFD_ROW_WPE))) row_kernel(const PassArgs args, const float2* __restrict__ tw) {
  __shared__ __align__(16) unsigned char lds[RowLds<L, GR, VAR, P>::bytes];
  row_body<L, GR, VAR, P>(args, tw, xcd_tile(blockIdx.x, args.total_tiles), lds, (int)threadIdx.x);
}

hipError_t launch_row_pass(int L, int G, int var, const PassArgs& a, const float2* tw, hipStream_t s) {
#define SFD_LAUNCH_V(l, g, p, v) \
  hipLaunchKernelGGL((row_kernel<l, g, v, p>), dim3(a.total_tiles), dim3(PassShape<l, g, p>::THREADS), 0, s, a, tw)
#define SFD_LAUNCH_ROW(l, g, p)                   \
  if (L == l && G == g) {                         \
    if (var == 2) SFD_LAUNCH_V(l, g, p, 2);       \
    else if (var == 3) SFD_LAUNCH_V(l, g, p, 3);  \
    else if (var == 1) SFD_LAUNCH_V(l, g, p, 1);  \
    else SFD_LAUNCH_V(l, g, p, 0);                \
    return hipGetLastError();                     \
  }
  SFD_ROW_SHAPES(SFD_LAUNCH_ROW)
#undef SFD_LAUNCH_ROW
#undef SFD_LAUNCH_V
  return hipErrorInvalidValue;
}

}  // namespace sfd
