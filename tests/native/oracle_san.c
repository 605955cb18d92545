/* The FP64 oracle under the address and undefined-behaviour sanitizers: every
 * entry point on small geometries whose delays run off both ends of the
 * records, all-pixel and listed-pixel calls, empty and out-of-range pixel
 * lists, and each argument rejected. Also a few identities that need no GPU:
 * DAS is linear in the record, the two DMAS forms agree, pDAS with p = 1 is
 * DAS. Prints "ok" lines; exits 1 at the first failed check. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/pwbf_oracle.c"

#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c);   \
      exit(1);                                                                \
    }                                                                         \
  } while (0)

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* xorshift64*, uniform in [-1, 1) */
  state ^= state >> 12;
  state ^= state << 25;
  state ^= state >> 27;
  return (double)((state * 2685821657736338717ull) >> 11) / 4503599627370496.0 - 1.0;
}

static int close_to(double a, double b, double rel) {
  return fabs(a - b) <= rel * (fabs(a) + fabs(b)) + 1e-300;
}

int main(void) {
  enum { NA = 3, NC = 8, NS = 40, NX = 6, NZ = 9 };
  double ex[NC], th[NA] = {-0.2, 0.0, 0.25}, t0[NA] = {0.0, 1e-7, -2e-7};
  for (int e = 0; e < NC; ++e) ex[e] = (e - 3.5) * 0.3e-3;
  ora_geom g;
  memset(&g, 0, sizeof g);
  g.n_angles = NA;
  g.n_channels = NC;
  g.n_samples = NS;
  g.elem_x = ex;
  g.angle = th;
  g.t0 = t0;
  g.c = 1540.0;
  g.fs = 20.8e6;
  g.nx = NX;
  g.nz = NZ;
  /* the grid reaches beyond the records at depth: delays past n_samples */
  g.x0 = -1.5e-3;
  g.dx = 0.6e-3;
  g.z0 = 0.2e-3;
  g.dz = 0.25e-3;
  g.f_number = 1.0;
  static double rf[NA * NC * NS], rf2[NA * NC * NS], qi[NA * NC * NS];
  for (int i = 0; i < NA * NC * NS; ++i) {
    rf[i] = urand();
    rf2[i] = 2.0 * rf[i];
    qi[i] = urand();
  }
  const int64_t total = NX * NZ;
  double a[NX * NZ], b[NX * NZ], c[NX * NZ], d[NX * NZ];
  for (int apod = 0; apod < 3; ++apod) {
    g.apod = apod;
    for (int angle = -1; angle < NA; ++angle) {
      CHECK(ora_das(&g, rf, angle, NULL, 0, a) == ORA_OK);
      CHECK(ora_das(&g, rf2, angle, NULL, 0, b) == ORA_OK);
      for (int64_t k = 0; k < total; ++k) CHECK(b[k] == 2.0 * a[k]);
      CHECK(ora_pdas(&g, rf, angle, 1.0, NULL, 0, c) == ORA_OK);
      for (int64_t k = 0; k < total; ++k) CHECK(close_to(c[k], a[k], 1e-12));
      CHECK(ora_dmas(&g, rf, angle, 0, NULL, 0, c) == ORA_OK);
      CHECK(ora_dmas(&g, rf, angle, 1, NULL, 0, d) == ORA_OK);
      for (int64_t k = 0; k < total; ++k) CHECK(close_to(c[k], d[k], 1e-9) || fabs(c[k]) < 1e-12);
      CHECK(ora_pdas(&g, rf, angle, 2.0, NULL, 0, c) == ORA_OK);
      CHECK(ora_iq(&g, rf, qi, 5.2e6, 0, angle, NULL, 0, c, d) == ORA_OK);
      CHECK(ora_iq(&g, rf, qi, 5.2e6, 1, angle, NULL, 0, c, d) == ORA_OK);
      /* listed pixels return the same values as the full image, in list order */
      const int64_t pix[4] = {total - 1, 0, 7, 7};
      double e4[4];
      CHECK(ora_das(&g, rf, angle, pix, 4, e4) == ORA_OK);
      for (int k = 0; k < 4; ++k) CHECK(e4[k] == a[pix[k]]);
      CHECK(ora_das(&g, rf, angle, pix, 0, e4) == ORA_OK); /* empty list */
    }
  }
  puts("ok entry points and identities");
  /* rejected arguments: nothing is written, nothing read out of bounds */
  const int64_t bad_hi[1] = {total}, bad_lo[1] = {-1};
  double o1[1] = {123.0};
  CHECK(ora_das(&g, rf, 0, bad_hi, 1, o1) == ORA_BAD && o1[0] == 123.0);
  CHECK(ora_das(&g, rf, 0, bad_lo, 1, o1) == ORA_BAD);
  CHECK(ora_dmas(&g, rf, 0, 2, NULL, 0, a) == ORA_BAD);
  CHECK(ora_dmas(&g, rf, NA, 0, NULL, 0, a) == ORA_BAD);
  CHECK(ora_pdas(&g, rf, 0, 0.5, NULL, 0, a) == ORA_BAD);
  CHECK(ora_pdas(&g, rf, 0, NAN, NULL, 0, a) == ORA_BAD);
  CHECK(ora_iq(&g, rf, qi, 5.2e6, 3, 0, NULL, 0, c, d) == ORA_BAD);
  CHECK(ora_das(&g, NULL, 0, NULL, 0, a) == ORA_BAD);
  CHECK(ora_das(&g, rf, -2, NULL, 0, a) == ORA_BAD);
  ora_geom h = g;
  h.n_angles = 0;
  CHECK(ora_das(&h, rf, -1, NULL, 0, a) == ORA_BAD);
  h = g;
  h.n_channels = 0;
  CHECK(ora_das(&h, rf, -1, NULL, 0, a) == ORA_BAD);
  puts("ok rejected arguments");
  puts("all ok");
  return 0;
}
