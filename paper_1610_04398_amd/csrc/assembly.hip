// The steps around the Poisson solve that read the gridded velocity.
//
// Pressure source (eq. PoissonFinal): at every grid node
//   f = -rho (u_x^2 + 2 u_y v_x + v_y^2) + rho lambda (d/dx[chi (u_s - u)] + d/dy[chi (v_s - v)]),
// the first term being grad u^T : grad u = u_{j,i} u_{i,j} written out in 2-D.
// Viscous forces (Sec. 2.3.2): dF = 2 mu D . n dS (eq. Fvisc) with
// D = (grad u + grad u^T) / 2 taken at the grid node nearest to each lifted
// surface point, summed per body (eq. FviscNet) and projected on the free
// stream (eq. CdNu).
//
// Derivatives are second-order central differences at interior nodes and
// second-order one-sided three-point differences on the first and last
// row/column (two nodes: the two-point difference; one node: 0).  Every
// expression keeps its written operation order (no contraction), so the
// results equal a plain evaluation of the same formulas bit for bit.  Node
// fields are row-major (a[j * nx + i]); one thread per node in row-major
// order, so all loads are coalesced and the rows a workgroup touches stay in
// L2.
#include <cmath>

#include "../../include/pp.h"
#include "internal.h"

namespace pp {

namespace {

// d a / d x at (i, j) (stride 1, n = nx) or d a / d y (stride nx, n = ny); k = i or j.
__device__ inline double diff1(const double* __restrict__ a, int64_t at, int64_t stride, int k, int n, double h) {
#pragma clang fp contract(off)
  const double two_h = 2.0 * h;
  if (n >= 3) {
    if (k == 0) return ((-3.0 * a[at] + 4.0 * a[at + stride]) - a[at + 2 * stride]) / two_h;
    if (k == n - 1) return ((3.0 * a[at] - 4.0 * a[at - stride]) + a[at - 2 * stride]) / two_h;
    return (a[at + stride] - a[at - stride]) / two_h;
  }
  if (n == 2) return k == 0 ? (a[at + stride] - a[at]) / h : (a[at] - a[at - stride]) / h;
  return 0.0;
}

// derivative of chi (s - a) at (i, j) along one axis, the product formed at each stencil node
__device__ inline double diff1_pen(const double* __restrict__ chi, const double* __restrict__ s,
                                   const double* __restrict__ a, int64_t at, int64_t stride, int k, int n,
                                   double h) {
#pragma clang fp contract(off)
  auto q = [&](int64_t o) { return chi[o] * (s[o] - a[o]); };
  const double two_h = 2.0 * h;
  if (n >= 3) {
    if (k == 0) return ((-3.0 * q(at) + 4.0 * q(at + stride)) - q(at + 2 * stride)) / two_h;
    if (k == n - 1) return ((3.0 * q(at) - 4.0 * q(at - stride)) + q(at - 2 * stride)) / two_h;
    return (q(at + stride) - q(at - stride)) / two_h;
  }
  if (n == 2) return k == 0 ? (q(at + stride) - q(at)) / h : (q(at) - q(at - stride)) / h;
  return 0.0;
}

__global__ __launch_bounds__(256) void k_source(const double* __restrict__ u, const double* __restrict__ v,
                                                const double* __restrict__ chi, const double* __restrict__ us,
                                                const double* __restrict__ vs, int nx, int ny, double h, double rho,
                                                double lam, double* __restrict__ f, int* __restrict__ flags) {
#pragma clang fp contract(off)
  const int64_t at = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (at >= (int64_t)nx * ny) return;
  const int j = (int)(at / nx), i = (int)(at - (int64_t)j * nx);
  const double ux = diff1(u, at, 1, i, nx, h), uy = diff1(u, at, nx, j, ny, h);
  const double vx = diff1(v, at, 1, i, nx, h), vy = diff1(v, at, nx, j, ny, h);
  double val = -rho * ((ux * ux + 2.0 * (uy * vx)) + vy * vy);
  if (chi) val = val + (rho * lam) * (diff1_pen(chi, us, u, at, 1, i, nx, h) + diff1_pen(chi, vs, v, at, nx, j, ny, h));
  if (!isfinite(val)) atomicOr(flags, kFlagNonFiniteSource);
  f[at] = val;
}

struct Comp {  // Neumaier-compensated sum
  double s = 0.0, c = 0.0;
  __device__ void add(double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
};

constexpr int kViscBlock = 256;

__global__ __launch_bounds__(kViscBlock) void k_viscous(const double* __restrict__ u, const double* __restrict__ v,
                                                         int nx, int ny, double x0, double y0, double h,
                                                         const double* __restrict__ lx, const double* __restrict__ ly,
                                                         const double* __restrict__ pnx, const double* __restrict__ pny,
                                                         const double* __restrict__ ds, const int64_t* __restrict__ seg,
                                                         double mu, double uxi, double uyi, double rho, double area,
                                                         double* __restrict__ dfx, double* __restrict__ dfy,
                                                         pp_force* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double rx[kViscBlock], ry[kViscBlock];
  const int64_t a = seg[blockIdx.x], b = seg[blockIdx.x + 1];
  Comp sx, sy;
  const double two_mu = 2.0 * mu;
  for (int64_t p = a + threadIdx.x; p < b; p += kViscBlock) {
    // nearest node: the node at the centre of the cell holding the point
    const double fi = floor((lx[p] - x0) / h), fj = floor((ly[p] - y0) / h);
    const int i = (int)fmin(fmax(fi, 0.0), (double)(nx - 1));
    const int j = (int)fmin(fmax(fj, 0.0), (double)(ny - 1));
    const int64_t at = (int64_t)j * nx + i;
    const double dux = diff1(u, at, 1, i, nx, h), duy = diff1(u, at, nx, j, ny, h);
    const double dvx = diff1(v, at, 1, i, nx, h), dvy = diff1(v, at, nx, j, ny, h);
    const double off = 0.5 * (duy + dvx);
    const double n0 = pnx[p], n1 = pny[p], d = ds[p];
    const double fx = (two_mu * (dux * n0 + off * n1)) * d;
    const double fy = (two_mu * (off * n0 + dvy * n1)) * d;
    if (dfx) dfx[p] = fx;
    if (dfy) dfy[p] = fy;
    sx.add(fx);
    sy.add(fy);
  }
  rx[threadIdx.x] = sx.s + sx.c;
  ry[threadIdx.x] = sy.s + sy.c;
  __syncthreads();
  for (int o = kViscBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      rx[threadIdx.x] += rx[threadIdx.x + o];
      ry[threadIdx.x] += ry[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double fx = rx[0], fy = ry[0];
    const double speed = sqrt(uxi * uxi + uyi * uyi);
    const double drag = (fx * uxi + fy * uyi) / speed;
    pp_force r;
    r.fx = fx;
    r.fy = fy;
    r.drag = drag;
    r.cd = 2.0 * drag / (rho * speed * speed * area);
    out[blockIdx.x] = r;
  }
}
}  // namespace

void pressure_source(const double* u, const double* v, const double* chi, const double* us, const double* vs, int nx,
                     int ny, double h, double rho, double lam, double* f, int* flags, hipStream_t s) {
  if (nx <= 0 || ny <= 0) return;
  const int64_t n = (int64_t)nx * ny;
  k_source<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(u, v, chi, us, vs, nx, ny, h, rho, lam, f, flags);
}

void viscous_forces(const double* u, const double* v, int nx, int ny, double x0, double y0, double h, const double* lx,
                    const double* ly, const double* pnx, const double* pny, const double* ds, int nseg,
                    const int64_t* seg, double mu, double uxi, double uyi, double rho, double area, double* dfx,
                    double* dfy, pp_force* out, hipStream_t s) {
  if (nseg <= 0) return;
  k_viscous<<<nseg, kViscBlock, 0, s>>>(u, v, nx, ny, x0, y0, h, lx, ly, pnx, pny, ds, seg, mu, uxi, uyi, rho, area,
                                        dfx, dfy, out);
}

}  // namespace pp
