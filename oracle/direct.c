/*
 * CPU oracle for the pressure-Poisson solve: the plain O(N*M) direct sum.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU path is
 * checked against; the product library never links or calls it.
 *
 * What it computes (Appendix A, eq. greenSum with the kernel of eq. green2D):
 *
 *     P(t_j) = sum_i G(t_j, s_i) f(s_i) h^2(s_i),   G(x, x') = (1/2pi) ln|x - x'|
 *
 * evaluated as (1/2pi) * sum_i w_i * 0.5 * ln(dx^2 + dy^2) with w_i = f_i h_i^2.
 * The sum is taken in FP64 in a fixed source order with Neumaier compensation;
 * targets are distributed over OpenMP threads with a static schedule, so the
 * result does not depend on the thread count.
 *
 * Self-interaction (a target that coincides with a source, r = 0, where the
 * kernel is singular) is not treated by the paper.  Two readings are offered:
 *   self_mode 0 (skip):    the coincident source contributes nothing;
 *   self_mode 1 (cellavg): it contributes w (ln h - kappa) / (2pi), the mean of
 *                          ln r over the h x h cell centred on the source,
 *                          kappa = 3/2 - pi/4 + ln(2)/2.
 * Coincidence means exact FP64 equality of both coordinates, with the grid
 * node coordinate computed as x0 + (i + 0.5) * h (no fused multiply-add).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>

#define ORACLE_KAPPA 1.0611754268825244 /* 3/2 - pi/4 + ln(2)/2 */
#define ORACLE_TWO_PI 6.283185307179586

/* Neumaier's improved Kahan summation: returns s + c at the end. */
typedef struct {
  double s, c;
} nsum;

static inline void nsum_add(nsum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

/*
 * Grid sources: f is ny*nx row-major, node (i, j) at (x0+(i+.5)h, y0+(j+.5)h).
 * Targets (tx[k], ty[k]), k < m.  out[k] receives P at target k.
 * Returns 0, or -1 on a bad argument.
 */
/* Threads of the target loop (0: the OpenMP default).  The result does not
 * depend on it: each target's sum runs in one thread in a fixed order. */
static int oracle_threads = 0;
void oracle_set_threads(int n) { oracle_threads = n > 0 ? n : 0; }
int oracle_get_threads(void) { return oracle_threads > 0 ? oracle_threads : omp_get_max_threads(); }

int oracle_direct_grid(int32_t nx, int32_t ny, double x0, double y0, double h, const double *f, int64_t m,
                       const double *tx, const double *ty, int32_t self_mode, double *out) {
  if (nx <= 0 || ny <= 0 || !(h > 0.0) || m < 0 || !f || (m > 0 && (!tx || !ty || !out))) return -1;
  if (self_mode != 0 && self_mode != 1) return -1;
  const double h2 = h * h;
  const double lnh = log(h);
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
  for (int64_t k = 0; k < m; ++k) {
    const double px = tx[k], py = ty[k];
    nsum acc = {0.0, 0.0};
    double self = 0.0;
    for (int32_t j = 0; j < ny; ++j) {
      const double sy = y0 + ((double)j + 0.5) * h;
      const double dy = py - sy;
      const double *frow = f + (size_t)j * (size_t)nx;
      for (int32_t i = 0; i < nx; ++i) {
        const double w = frow[i] * h2;
        if (w == 0.0) continue;
        const double sx = x0 + ((double)i + 0.5) * h;
        const double dx = px - sx;
        if (dx == 0.0 && dy == 0.0) {
          if (self_mode == 1) self += w * (lnh - ORACLE_KAPPA);
          continue;
        }
        nsum_add(&acc, w * 0.5 * log(dx * dx + dy * dy));
      }
    }
    out[k] = ((acc.s + acc.c) + self) / ORACLE_TWO_PI;
  }
  return 0;
}

/*
 * Scattered sources with per-source weight w_i = f_i h_i^2 (eq. greenSum with a
 * spatially varying cell area).  A coincident source is skipped.
 */
int oracle_direct_points(int64_t n, const double *sx, const double *sy, const double *w, int64_t m,
                         const double *tx, const double *ty, double *out) {
  if (n < 0 || m < 0 || (n > 0 && (!sx || !sy || !w)) || (m > 0 && (!tx || !ty || !out))) return -1;
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
  for (int64_t k = 0; k < m; ++k) {
    const double px = tx[k], py = ty[k];
    nsum acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
      if (w[i] == 0.0) continue;
      const double dx = px - sx[i];
      const double dy = py - sy[i];
      if (dx == 0.0 && dy == 0.0) continue;
      nsum_add(&acc, w[i] * 0.5 * log(dx * dx + dy * dy));
    }
    out[k] = (acc.s + acc.c) / ORACLE_TWO_PI;
  }
  return 0;
}
