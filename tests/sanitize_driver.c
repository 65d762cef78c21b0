/* Drives every entry point of the C oracle on small and ragged grids, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).  Test
 * infrastructure: it links the oracle source directly.  Exit status 0 when every call returned
 * what it should; the sanitizers abort on any invalid access or undefined behaviour. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  double r, R;
  int32_t n_theta, n_phi;
  double A, kappa, M, tau, dt;
  uint32_t flags;
} tlbref_params;
typedef struct tlbref_grid tlbref_grid;

int tlbref_create(const tlbref_params* p, tlbref_grid** out);
void tlbref_destroy(tlbref_grid* g);
int tlbref_set_state(tlbref_grid* g, const double* f, const double* phi, const double* n,
                     const double* ut, const double* up);
int tlbref_get_state(tlbref_grid* g, double* f, double* phi);
int tlbref_step_n(tlbref_grid* g, int64_t nsteps);
int tlbref_get_moments(tlbref_grid* g, double* n, double* ut, double* up, double* phi,
                       double* mu);
int tlbref_invariants(tlbref_grid* g, double out[3]);
int tlbref_rhs_terms(tlbref_grid* g, const double* f, const double* phi, double* Lf,
                     double* Lphi, double* adv, double* frc, double* con, double* bgk,
                     double* mu, double* lap, double* Fth, double* Fph);
int tlbref_geometry(tlbref_grid* g, double* J, double* Jp, double* Jm, double* G);
int tlbref_diagnostics(tlbref_grid* g, double out[2], double* phi_avg, double* p_avg);
void tlbref_velocity_set(double v[4], double w[4], double K[16], double Kt[16]);
double tlbref_uw5_face(const double h[5]);
double tlbref_weno5_face(const double h[5], double eps);
int64_t tlbref_steps(const tlbref_grid* g);

static int failures = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static double* alloc(size_t n) {
  double* p = calloc(n, sizeof(double));
  if (!p) abort();
  return p;
}

/* one grid through the whole interface */
static void exercise(int nt, int np, uint32_t flags) {
  tlbref_params p = {1.0, 2.5, nt, np, 0.5, 2e-3, 0.05, 0.3, 2e-4, flags};
  tlbref_grid* g = NULL;
  CHECK(tlbref_create(&p, &g) == 0 && g);
  if (!g) return;
  const size_t nn = (size_t)nt * np;
  double *phi = alloc(nn), *n = alloc(nn), *ut = alloc(nn), *up = alloc(nn);
  double *f = alloc(16 * nn), *mu = alloc(nn);
  for (size_t x = 0; x < nn; ++x) {
    phi[x] = 0.5 * sin(0.37 * (double)x);
    n[x] = 1.0 + 0.05 * cos(0.11 * (double)x);
    ut[x] = 0.02 * sin(0.05 * (double)x);
    up[x] = -0.03 * cos(0.07 * (double)x);
  }
  CHECK(tlbref_set_state(g, NULL, phi, n, ut, up) == 0);
  CHECK(tlbref_step_n(g, 20) == 0);
  CHECK(tlbref_steps(g) == 20);
  CHECK(tlbref_get_state(g, f, phi) == 0);
  CHECK(tlbref_get_moments(g, n, ut, up, phi, mu) == 0);
  double inv[3];
  CHECK(tlbref_invariants(g, inv) == 0 && inv[2] == 0.0);
  double d[2];
  double *pa = alloc(nt), *pp = alloc(nt);
  CHECK(tlbref_diagnostics(g, d, pa, pp) == 0);
  double *J = alloc(nt), *Jp = alloc(nt), *Jm = alloc(nt), *G = alloc(nt);
  CHECK(tlbref_geometry(g, J, Jp, Jm, G) == 0);
  double *Lf = alloc(16 * nn), *adv = alloc(16 * nn), *frc = alloc(16 * nn);
  double *con = alloc(16 * nn), *bgk = alloc(16 * nn);
  double *Lphi = alloc(nn), *mu2 = alloc(nn), *lap = alloc(nn), *Fth = alloc(nn), *Fph = alloc(nn);
  CHECK(tlbref_rhs_terms(g, f, phi, Lf, Lphi, adv, frc, con, bgk, mu2, lap, Fth, Fph) == 0);
  /* resume from the checkpoint, then a non-finite value is detected */
  CHECK(tlbref_set_state(g, f, phi, NULL, NULL, NULL) == 0);
  CHECK(tlbref_step_n(g, 3) == 0);
  phi[nn / 2] = NAN;
  CHECK(tlbref_set_state(g, f, phi, NULL, NULL, NULL) == 0);
  CHECK(tlbref_invariants(g, inv) != 0 && inv[2] >= 1.0);
  tlbref_destroy(g);
  free(phi); free(n); free(ut); free(up); free(f); free(mu); free(pa); free(pp);
  free(J); free(Jp); free(Jm); free(G); free(Lf); free(adv); free(frc); free(con); free(bgk);
  free(Lphi); free(mu2); free(lap); free(Fth); free(Fph);
}

int main(void) {
  const int shapes[][2] = {{24, 40}, {37, 150}, {9, 70}, {6, 1}, {3, 5}, {1, 9}};
  const uint32_t flag_sets[] = {0u, 1u, 2u, 8u};
  for (size_t i = 0; i < sizeof(shapes) / sizeof(shapes[0]); ++i)
    for (size_t k = 0; k < sizeof(flag_sets) / sizeof(flag_sets[0]); ++k)
      exercise(shapes[i][0], shapes[i][1], flag_sets[k]);
  /* invalid parameters are refused without touching anything */
  tlbref_grid* g = NULL;
  tlbref_params bad = {0.0, 2.5, 8, 8, 0.5, 2e-3, 0.05, 0.3, 2e-4, 0u};
  CHECK(tlbref_create(&bad, &g) != 0 && g == NULL);
  bad.r = 1.0;
  bad.R = 0.5;
  CHECK(tlbref_create(&bad, &g) != 0 && g == NULL);
  CHECK(tlbref_create(NULL, &g) != 0);
  tlbref_destroy(NULL);
  double v[4], w[4], K[16], Kt[16], h[5] = {0.1, 0.2, 0.3, 0.25, 0.2};
  tlbref_velocity_set(v, w, K, Kt);
  CHECK(fabs(tlbref_uw5_face(h) - tlbref_weno5_face(h, 1e30)) < 1e-12);
  if (failures) fprintf(stderr, "%d checks failed\n", failures);
  else printf("all oracle entry points ran clean\n");
  return failures ? 1 : 0;
}
