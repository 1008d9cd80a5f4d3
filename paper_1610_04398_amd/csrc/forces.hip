// Pressure forces on body surfaces (Sec. 2.3.1): the pointwise force
// dF_P = -P n dS (eq. Fpress) of every surface panel, its closed surface
// integral F_P (eq. FpressNet) per body, and the drag along the free stream
// with its coefficient 2 Drag / (rho |U|^2 A) (eq. CdP).
//
// One workgroup per body (segment of consecutive panels): thread i takes panels
// i, i + 256, ... in order with a compensated FP64 sum, then the 256 partial
// sums are combined by a fixed tree in LDS, so the result does not depend on
// the hardware's scheduling.
#include <cmath>

#include "../../include/pp.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kForceBlock = 256;

struct Comp {  // Neumaier-compensated sum
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
};

__global__ __launch_bounds__(kForceBlock) void k_forces(const double* __restrict__ p, const double* __restrict__ nx,
                                                         const double* __restrict__ ny, const double* __restrict__ ds,
                                                         const int64_t* __restrict__ seg, double ux, double uy,
                                                         double rho, double area, double* __restrict__ dfx,
                                                         double* __restrict__ dfy, pp_force* __restrict__ out) {
  __shared__ double rx[kForceBlock], ry[kForceBlock];
  const int64_t a = seg[blockIdx.x], b = seg[blockIdx.x + 1];
  Comp sx, sy;
  for (int64_t j = a + threadIdx.x; j < b; j += kForceBlock) {
    const double pj = -p[j], dsj = ds[j];
    const double fx = (pj * nx[j]) * dsj, fy = (pj * ny[j]) * dsj;
    if (dfx) dfx[j] = fx;
    if (dfy) dfy[j] = fy;
    sx.add(fx);
    sy.add(fy);
  }
  rx[threadIdx.x] = sx.s + sx.c;
  ry[threadIdx.x] = sy.s + sy.c;
  __syncthreads();
  for (int o = kForceBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      rx[threadIdx.x] += rx[threadIdx.x + o];
      ry[threadIdx.x] += ry[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double fx = rx[0], fy = ry[0];
    const double speed = sqrt(ux * ux + uy * uy);
    const double drag = (fx * ux + fy * uy) / speed;
    pp_force f;
    f.fx = fx;
    f.fy = fy;
    f.drag = drag;
    f.cd = 2.0 * drag / (rho * speed * speed * area);
    out[blockIdx.x] = f;
  }
}
}  // namespace

void surface_forces(const double* p, const double* nx, const double* ny, const double* ds, int nseg,
                    const int64_t* seg, double ux, double uy, double rho, double area, double* dfx, double* dfy,
                    pp_force* out, hipStream_t s) {
  if (nseg <= 0) return;
  k_forces<<<nseg, kForceBlock, 0, s>>>(p, nx, ny, ds, seg, ux, uy, rho, area, dfx, dfy, out);
}

}  // namespace pp
