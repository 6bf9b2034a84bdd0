/* A plain C caller of the library: only include/ttn.h and the HIP runtime's
 * C API.  "cpu": argument and configuration errors that return before any
 * device call.  "gpu": a transverse-field Ising chain (L = 32, h = 1,
 * chi = 6, float64, seeded isometries) initialised, swept twice with the
 * paper's sweep and once with the grouped sweep; prints the energies, one per
 * line, then the sum of the local energies of the final state, for the caller
 * to compare.  Exit status 0 on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "ttn.h"

static void tfim(double h1[4], double A[4], double B[4], double field) {
  /* one-site term -h X, bond term -Z Z as A = Z on site j, B = -Z on site j+1 */
  h1[0] = 0.0; h1[1] = -field; h1[2] = -field; h1[3] = 0.0;
  A[0] = 1.0; A[1] = 0.0; A[2] = 0.0; A[3] = -1.0;
  B[0] = -1.0; B[1] = 0.0; B[2] = 0.0; B[3] = 1.0;
}

static void config(ttn_config* c, const double* h1, const double* A, const double* B) {
  memset(c, 0, sizeof *c);
  c->L = 32;
  c->d = 2;
  c->chi = 6;
  c->D = 1;
  c->h1 = h1;
  c->A = A;
  c->B = B;
  c->shift = NAN; /* library default */
  c->ly = 1;
  c->precision = TTN_FP64;
  c->seed = 7;
}

static int fail(const char* what, ttn_status st) {
  fprintf(stderr, "%s: status %d (%s)\n", what, st, ttn_last_error());
  return 1;
}

static int cpu_checks(void) {
  double h1[4], A[4], B[4];
  tfim(h1, A, B, 1.0);
  ttn_config c;
  config(&c, h1, A, B);
  size_t bytes = 0;
  ttn_status st = ttn_workspace_bytes(&c, 1, &bytes);
  if (st != TTN_OK || bytes == 0) return fail("workspace size", st);
  c.L = 24; /* not a power of two */
  if ((st = ttn_workspace_bytes(&c, 1, &bytes)) != TTN_EINVAL) return fail("L = 24 accepted", st);
  if (ttn_last_error()[0] == '\0') return fail("no error text", st);
  c.L = 32;
  if ((st = ttn_workspace_bytes(&c, 0, &bytes)) != TTN_EINVAL) return fail("empty batch accepted", st);
  if ((st = ttn_sweep(NULL, 1, 0)) != TTN_EINVAL) return fail("null handle sweep", st);
  if ((st = ttn_sweep_grouped(NULL, 1, 2, 0)) != TTN_EINVAL) return fail("null handle grouped sweep", st);
  double e;
  if ((st = ttn_energy(NULL, &e)) != TTN_EINVAL) return fail("null handle energy", st);
  double site[32], bond[32];
  if ((st = ttn_positions_bytes(NULL, 0, &bytes)) != TTN_EINVAL) return fail("null handle positions bytes", st);
  if ((st = ttn_local_energies(NULL, 0, NULL, 0, site, bond)) != TTN_EINVAL) return fail("null handle local energies", st);
  printf("cpu checks passed\n");
  return 0;
}

static int gpu_run(void) {
  double h1[4], A[4], B[4];
  tfim(h1, A, B, 1.0);
  ttn_config c;
  config(&c, h1, A, B);
  size_t bytes = 0;
  ttn_status st = ttn_workspace_bytes(&c, 1, &bytes);
  if (st != TTN_OK) return fail("workspace size", st);
  void* ws = NULL;
  if (hipMalloc(&ws, bytes) != hipSuccess) {
    fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
    return 1;
  }
  ttn_handle h = NULL;
  int rc = 1;
  double e0, e1, e2, total = 0.0;
  double site[32], bond[32];
  size_t pbytes = 0;
  void* work = NULL;
  if ((st = ttn_init(&c, 1, ws, bytes, NULL, &h)) != TTN_OK) { fail("init", st); goto out; }
  if ((st = ttn_energy(h, &e0)) < 0) { fail("energy", st); goto out; }
  if ((st = ttn_sweep(h, 2, 0)) < 0) { fail("sweep", st); goto out; }
  if ((st = ttn_energy(h, &e1)) < 0) { fail("energy", st); goto out; }
  if ((st = ttn_sweep_grouped(h, 1, 2, 0)) < 0) { fail("grouped sweep", st); goto out; }
  if ((st = ttn_energy(h, &e2)) < 0) { fail("energy", st); goto out; }
  if (ttn_bond_dim(h, 0, 1) != 4) { fprintf(stderr, "bond dimension of level 1\n"); goto out; }
  /* local energies in a work buffer of the minimum size */
  if ((st = ttn_positions_bytes(h, 0, &pbytes)) != TTN_OK) { fail("positions bytes", st); goto out; }
  if (hipMalloc(&work, pbytes) != hipSuccess) { fprintf(stderr, "hipMalloc of %zu bytes failed\n", pbytes); goto out; }
  if ((st = ttn_local_energies(h, 0, work, pbytes, site, bond)) != TTN_OK) { fail("local energies", st); goto out; }
  for (int j = 0; j < 32; ++j) total += site[j] + bond[j];
  printf("%.17g\n%.17g\n%.17g\n%.17g\n", e0, e1, e2, total);
  rc = 0;
out:
  if (h) ttn_free(h);
  if (work) (void)hipFree(work);
  (void)hipFree(ws);
  return rc;
}

int main(int argc, char** argv) {
  if (argc > 1 && strcmp(argv[1], "gpu") == 0) return gpu_run();
  return cpu_checks();
}
