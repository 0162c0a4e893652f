/*
 * oracle.c -- plain CPU reference for iterated, out-of-place Jacobi stencil sweeps.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. The product path never calls it and
 * shares no source with it.
 *
 * What it computes (paper, Section 2.1 "Stencils", Listings 1-3): each time step
 * replaces every interior cell by a weighted sum of its neighbours at the
 * previous step,
 *
 *     U^s(i) = sum_{p in P} w_p * U^{s-1}(i + p),      s = 1..T,
 *
 * reading only U^{s-1} (out-of-place, Jacobi style). The listings index in[i-1]
 * at the first cell without saying what lies there; this reference takes the
 * reading of a Dirichlet halo of width r that is held at its initial values for
 * every step (cells outside the interior never change).
 *
 * Layout: a row-major padded array with extents n_j + 2r per dimension,
 * slowest dimension first, x fastest. The coefficient array is the dense
 * (2r+1)^ndim box, row-major with the slowest offset first; an entry that is
 * exactly 0.0 is an absent point (no term).
 *
 * Summation order: terms are accumulated in the dense box order (offsets
 * sorted lexicographically, slowest axis first), starting from +0.0, with one
 * fused multiply-add per term. That fixes the rounding of every result.
 *
 * No tiling, no temporal blocking: one full sweep per step, then swap.
 * OpenMP splits the interior rows across threads; each cell is computed by
 * exactly the same operations regardless of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_TAPS 729 /* (2*4+1)^3 */

typedef struct {
  int64_t off; /* linear offset in the padded array */
  double w;
} tap_t;

/* Collect the non-zero taps in dense-box order. Returns the number of taps. */
static int collect_taps(int ndim, int r, const int64_t *pext, const double *coeffs,
                        tap_t *taps) {
  int side = 2 * r + 1;
  int count = 1;
  for (int d = 0; d < ndim; ++d) count *= side;
  int k = 0;
  for (int idx = 0; idx < count; ++idx) {
    double w = coeffs[idx];
    if (w == 0.0) continue;
    /* decompose idx into per-axis offsets, slowest axis first */
    int rem = idx;
    int64_t off = 0;
    int64_t stride = 1;
    for (int d = ndim - 1; d >= 0; --d) {
      int p = rem % side - r;
      rem /= side;
      off += (int64_t)p * stride;
      stride *= pext[d];
    }
    taps[k].off = off;
    taps[k].w = w;
    ++k;
  }
  return k;
}

static int check_args(int ndim, const int64_t *n, int r, int64_t T) {
  if (ndim < 1 || ndim > 3) return -1;
  if (r < 0 || r > 4) return -1;
  if (T < 0) return -1;
  for (int d = 0; d < ndim; ++d)
    if (n[d] < 1) return -1;
  return 0;
}

/*
 * Double precision sweep. `in`, `out` and `work` each hold the whole padded
 * array. `in` is read only; the result U^T (halo included) lands in `out`.
 * `work` is scratch of the same size. Returns 0, or -1 on bad arguments.
 */
int oracle_sweep_f64(int ndim, const int64_t *n, int r, const double *coeffs, int64_t T,
                     const double *in, double *out, double *work, int nthreads) {
  if (check_args(ndim, n, r, T)) return -1;
  int64_t pext[3] = {1, 1, 1};
  int64_t total = 1;
  for (int d = 0; d < ndim; ++d) {
    pext[d] = n[d] + 2 * r;
    total *= pext[d];
  }
  tap_t taps[ORACLE_MAX_TAPS];
  int k = collect_taps(ndim, r, pext, coeffs, taps);

  memcpy(out, in, (size_t)total * sizeof(double));
  memcpy(work, in, (size_t)total * sizeof(double));
  double *src = out, *dst = work;

  /* interior index ranges, padded to three dimensions */
  int64_t lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, ext[3] = {1, 1, 1};
  for (int d = 0; d < ndim; ++d) {
    int e = 3 - ndim + d;
    lo[e] = r;
    hi[e] = n[d] + r;
    ext[e] = pext[d];
  }
  if (nthreads < 1) nthreads = 1;

  for (int64_t s = 0; s < T; ++s) {
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int64_t z = lo[0]; z < hi[0]; ++z) {
      for (int64_t y = lo[1]; y < hi[1]; ++y) {
        int64_t row = (z * ext[1] + y) * ext[2];
        /* every cell of the row accumulates its terms in tap order */
        double *acc = dst + row;
        for (int64_t x = lo[2]; x < hi[2]; ++x) acc[x] = 0.0;
        for (int q = 0; q < k; ++q) {
          const double w = taps[q].w;
          const double *nb = src + row + taps[q].off;
          for (int64_t x = lo[2]; x < hi[2]; ++x) acc[x] = fma(w, nb[x], acc[x]);
        }
      }
    }
    double *t = src;
    src = dst;
    dst = t;
  }
  if (src != out) memcpy(out, src, (size_t)total * sizeof(double));
  return 0;
}

/*
 * Single precision twin: the same sweep with float storage, coefficients
 * rounded once to float (round to nearest even), and fmaf.
 */
int oracle_sweep_f32(int ndim, const int64_t *n, int r, const double *coeffs, int64_t T,
                     const float *in, float *out, float *work, int nthreads) {
  if (check_args(ndim, n, r, T)) return -1;
  int64_t pext[3] = {1, 1, 1};
  int64_t total = 1;
  for (int d = 0; d < ndim; ++d) {
    pext[d] = n[d] + 2 * r;
    total *= pext[d];
  }
  tap_t taps[ORACLE_MAX_TAPS];
  int k = collect_taps(ndim, r, pext, coeffs, taps);
  float wf[ORACLE_MAX_TAPS];
  int64_t offs[ORACLE_MAX_TAPS];
  for (int q = 0; q < k; ++q) {
    wf[q] = (float)taps[q].w;
    offs[q] = taps[q].off;
  }

  memcpy(out, in, (size_t)total * sizeof(float));
  memcpy(work, in, (size_t)total * sizeof(float));
  float *src = out, *dst = work;

  int64_t lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, ext[3] = {1, 1, 1};
  for (int d = 0; d < ndim; ++d) {
    int e = 3 - ndim + d;
    lo[e] = r;
    hi[e] = n[d] + r;
    ext[e] = pext[d];
  }
  if (nthreads < 1) nthreads = 1;

  for (int64_t s = 0; s < T; ++s) {
#pragma omp parallel for collapse(2) num_threads(nthreads) schedule(static)
    for (int64_t z = lo[0]; z < hi[0]; ++z) {
      for (int64_t y = lo[1]; y < hi[1]; ++y) {
        int64_t row = (z * ext[1] + y) * ext[2];
        float *acc = dst + row;
        for (int64_t x = lo[2]; x < hi[2]; ++x) acc[x] = 0.0f;
        for (int q = 0; q < k; ++q) {
          const float w = wf[q];
          const float *nb = src + row + offs[q];
          for (int64_t x = lo[2]; x < hi[2]; ++x) acc[x] = fmaf(w, nb[x], acc[x]);
        }
      }
    }
    float *t = src;
    src = dst;
    dst = t;
  }
  if (src != out) memcpy(out, src, (size_t)total * sizeof(float));
  return 0;
}
