/* Pulse accumulation for the synthetic RF generator.
 *
 * Adds, for every element row and scatterer, amp * p(n/fs - t) to the samples
 * n within the pulse support, where p(t) = exp(-t^2 / (2 sigma^2)) cos(2 pi f0 t)
 * is truncated at |t| <= trunc. Arrival times t come from the caller.
 *
 * The Gaussian and the cosine are evaluated through the factorisation
 *   dt = k/fs + d, d = nc/fs - t,
 *   exp(-dt^2/2s^2) = exp(-d^2/2s^2) * exp(-k d/(fs s^2)) * exp(-k^2/(2 fs^2 s^2)),
 *   cos(w dt)       = cos(w d) cos(w k/fs) - sin(w d) sin(w k/fs),
 * so each (row, scatterer) costs four transcendentals instead of two per tap.
 * Rows are independent; each row is summed by one thread in scatterer order,
 * so the result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define MAXTAPS 257

void sim_accumulate(int32_t n_rows, int32_t n_samp, int64_t n_scat, const double *t,
                    const double *amp, double fs, double f0, double sigma, double trunc,
                    double *rf) {
  int half = (int)ceil(trunc * fs);
  if (half > (MAXTAPS - 1) / 2) half = (MAXTAPS - 1) / 2;
  const double two_pi = 6.283185307179586476925286766559;
  double gk[MAXTAPS], ck[MAXTAPS], sk[MAXTAPS];
  for (int k = -half; k <= half; ++k) {
    double tk = k / fs;
    gk[k + half] = exp(-0.5 * (tk / sigma) * (tk / sigma));
    ck[k + half] = cos(two_pi * f0 * tk);
    sk[k + half] = sin(two_pi * f0 * tk);
  }
  const double inv_fs = 1.0 / fs;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t r = 0; r < n_rows; ++r) {
    double *row = rf + (int64_t)r * n_samp;
    const double *tr = t + (int64_t)r * n_scat;
    for (int64_t s = 0; s < n_scat; ++s) {
      double ts = tr[s];
      double nc = rint(ts * fs);
      double d = nc * inv_fs - ts;
      double alpha = amp[s] * exp(-0.5 * (d / sigma) * (d / sigma));
      double ratio = exp(-d / (fs * sigma * sigma));
      double cp = cos(two_pi * f0 * d), sp = sin(two_pi * f0 * d);
      int64_t n0 = (int64_t)nc;
      /* positive taps */
      double rk = 1.0;
      for (int k = 0; k <= half; ++k) {
        int64_t n = n0 + k;
        double dt = d + k * inv_fs;
        if (n >= 0 && n < n_samp && fabs(dt) <= trunc)
          row[n] += alpha * rk * gk[k + half] * (cp * ck[k + half] - sp * sk[k + half]);
        rk *= ratio;
      }
      rk = 1.0 / ratio;
      for (int k = -1; k >= -half; --k) {
        int64_t n = n0 + k;
        double dt = d + k * inv_fs;
        if (n >= 0 && n < n_samp && fabs(dt) <= trunc)
          row[n] += alpha * rk * gk[k + half] * (cp * ck[k + half] - sp * sk[k + half]);
        rk /= ratio;
      }
    }
  }
}
