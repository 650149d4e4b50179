/* A plain C caller of libcem.so: no PyTorch and no C++ in the process.
 *
 * Usage: cube_force DIR N_NODES N_TETS N_FACES STEPS E NU RHO
 *
 * Reads from DIR (raw little-endian arrays):
 *   X.bin    double [N_NODES][3]   node coordinates (m)
 *   tets.bin int32  [N_TETS][4]    tet node ids
 *   u.bin    double [N_NODES][3]   a displacement field (m)
 *   tri.bin  int32  [N_FACES][3]   loaded boundary triangles
 *   trac.bin double [N_FACES][3]   their tractions (Pa)
 * Writes to DIR:
 *   f.bin    double [N_NODES][3]   internal force of u on the uploaded mesh
 *   us.bin   double [N_NODES][3]   displacement after STEPS steps from rest at
 *                                  half the critical step, traction applied at once
 * and prints the critical step and the energies of the run.  Exit status 0 on
 * success, 1 on a usage or file error, 2 on a library error (its message is
 * printed). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cem.h"

static void* read_file(const char* dir, const char* name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* fp = fopen(path, "rb");
  if (!fp) return NULL;
  void* p = malloc(bytes ? bytes : 1);
  size_t got = p ? fread(p, 1, bytes, fp) : 0;
  fclose(fp);
  if (got != bytes) {
    free(p);
    return NULL;
  }
  return p;
}

static int write_file(const char* dir, const char* name, const void* p, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* fp = fopen(path, "wb");
  if (!fp) return 1;
  size_t put = fwrite(p, 1, bytes, fp);
  return fclose(fp) != 0 || put != bytes;
}

static int fail(cem_ctx* ctx, const char* call, int rc) {
  fprintf(stderr, "%s returned %d: %s\n", call, rc, ctx ? cem_last_error(ctx) : "");
  if (ctx) cem_destroy(ctx);
  return 2;
}

int main(int argc, char** argv) {
  if (argc != 9) {
    fprintf(stderr, "usage: %s DIR N_NODES N_TETS N_FACES STEPS E NU RHO\n", argv[0]);
    return 1;
  }
  const char* dir = argv[1];
  const int n = atoi(argv[2]), nt = atoi(argv[3]), nf = atoi(argv[4]), steps = atoi(argv[5]);
  const cem_material mat = {atof(argv[6]), atof(argv[7]), atof(argv[8]), INFINITY};
  const size_t v3 = sizeof(double) * 3 * (size_t)n;
  double* X = read_file(dir, "X.bin", v3);
  int32_t* tets = read_file(dir, "tets.bin", sizeof(int32_t) * 4 * (size_t)nt);
  double* u = read_file(dir, "u.bin", v3);
  int32_t* tri = read_file(dir, "tri.bin", sizeof(int32_t) * 3 * (size_t)nf);
  double* trac = read_file(dir, "trac.bin", sizeof(double) * 3 * (size_t)nf);
  double* f = malloc(v3);
  double* us = malloc(v3);
  if (!X || !tets || !u || !tri || !trac || !f || !us) {
    fprintf(stderr, "cannot read the inputs in %s\n", dir);
    return 1;
  }

  cem_options opt;
  memset(&opt, 0, sizeof opt);
  opt.device = 0;
  opt.stream = NULL;  /* the context creates its own stream */
  opt.precision = CEM_FP64;
  opt.split_mode = CEM_PHANTOM;
  opt.gsig = CEM_GSIG_PRINCIPAL;
  opt.max_splits = 64;
  opt.graph_steps = 0;

  cem_ctx* ctx = NULL;
  int rc = cem_create(&opt, &ctx);
  if (rc) return fail(ctx, "cem_create", rc);
  if ((rc = cem_upload_mesh(ctx, n, X, nt, tets, &mat))) return fail(ctx, "cem_upload_mesh", rc);
  if ((rc = cem_internal_force(ctx, u, f))) return fail(ctx, "cem_internal_force", rc);

  double dtc = 0.0;
  if ((rc = cem_set_traction(ctx, nf, tri, trac, 0.0))) return fail(ctx, "cem_set_traction", rc);
  if ((rc = cem_critical_dt(ctx, &dtc))) return fail(ctx, "cem_critical_dt", rc);
  if ((rc = cem_set_dt(ctx, 0.5 * dtc))) return fail(ctx, "cem_set_dt", rc);
  if ((rc = cem_step(ctx, steps))) return fail(ctx, "cem_step", rc);
  int32_t nn = 0;
  if ((rc = cem_get_state(ctx, us, NULL, NULL, &nn))) return fail(ctx, "cem_get_state", rc);
  cem_energy e;
  if ((rc = cem_read_energy(ctx, &e))) return fail(ctx, "cem_read_energy", rc);
  cem_destroy(ctx);

  if (nn != n || write_file(dir, "f.bin", f, v3) || write_file(dir, "us.bin", us, v3)) {
    fprintf(stderr, "cannot write the outputs in %s (nodes %d)\n", dir, nn);
    return 1;
  }
  printf("dt_crit %.17g steps %lld KE %.17g SE %.17g Wext %.17g\n", dtc, (long long)e.step, e.KE,
         e.SE, e.Wext);
  free(X); free(tets); free(u); free(tri); free(trac); free(f); free(us);
  return 0;
}
