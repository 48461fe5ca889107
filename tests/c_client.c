/* A plain C client of the mfh C ABI (include/mfh.h), no Python or torch:
 * builds a 3-D Q2 problem with a two-level hierarchy and one stiff sphere,
 * clamped at the bottom and top faces, sets the displacement read from a
 * file, applies the matrix-free tangent (Sec. 4) and solves K x = b with the
 * multigrid-preconditioned CG (Sec. 6-7), and writes K x and the solution.
 *
 *   c_client N u.bin x.bin y.bin z.bin
 *
 * N cells per direction (even); u.bin, x.bin: n_dofs doubles (the DoF
 * numbering of the ABI); writes y = K_c x and z = K_c^-1 x, and prints the
 * CG iteration count and relative residual.  Exit code 0 on success. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "mfh.h"

#define HIP_OK(call)                                                  \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) {                                           \
      fprintf(stderr, "HIP error %s at %s\n", hipGetErrorString(e_), #call); \
      return 2;                                                       \
    }                                                                 \
  } while (0)

#define MFH_OK(call, P)                                               \
  do {                                                                \
    mfh_status s_ = (call);                                           \
    if (s_ != MFH_OK) {                                               \
      fprintf(stderr, "mfh error %d at %s: %s\n", (int)s_, #call, mfh_last_error(P)); \
      return 3;                                                       \
    }                                                                 \
  } while (0)

static int read_vec(const char* path, double* v, long long n) {
  FILE* f = fopen(path, "rb");
  if (!f) return 0;
  size_t got = fread(v, sizeof(double), (size_t)n, f);
  fclose(f);
  return got == (size_t)n;
}

static int write_vec(const char* path, const double* v, long long n) {
  FILE* f = fopen(path, "wb");
  if (!f) return 0;
  size_t put = fwrite(v, sizeof(double), (size_t)n, f);
  fclose(f);
  return put == (size_t)n;
}

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s N u.bin x.bin y.bin z.bin\n", argv[0]);
    return 1;
  }
  const double mu[2] = {1.0, 100.0}, lambda[2] = {1.5, 150.0};
  const double sphere[5] = {0.5, 0.5, 0.5, 0.2, 1.0};   /* centre, radius, material id */
  mfh_desc d;
  mfh_desc_defaults(&d);
  d.dim = 3;
  d.n_cells = atoi(argv[1]);
  d.degree = 2;
  d.n_levels = 2;
  d.n_materials = 2;
  d.mu = mu;
  d.lambda = lambda;
  d.n_inclusions = 1;
  d.inclusions = sphere;
  /* bit (2 * axis + side) * dim + component: faces z = 0 and z = 1, all components */
  for (int side = 0; side < 2; ++side)
    for (int c = 0; c < 3; ++c) d.dirichlet_mask |= 1u << ((2 * 2 + side) * 3 + c);
  d.qp_policy = MFH_QP_CACHE_T2;

  size_t bytes = 0;
  MFH_OK(mfh_workspace_size(&d, &bytes), NULL);
  void* ws = NULL;
  HIP_OK(hipMalloc(&ws, bytes));
  mfh_problem* P = NULL;
  MFH_OK(mfh_create(&d, ws, bytes, NULL, &P), NULL);
  long long n = 0;
  MFH_OK(mfh_n_dofs(P, d.n_levels - 1, &n), P);

  double* h = (double*)malloc((size_t)n * sizeof(double));
  double *u = NULL, *x = NULL, *y = NULL, *z = NULL;
  HIP_OK(hipMalloc((void**)&u, (size_t)n * sizeof(double)));
  HIP_OK(hipMalloc((void**)&x, (size_t)n * sizeof(double)));
  HIP_OK(hipMalloc((void**)&y, (size_t)n * sizeof(double)));
  HIP_OK(hipMalloc((void**)&z, (size_t)n * sizeof(double)));
  if (!h || !read_vec(argv[2], h, n)) { fprintf(stderr, "cannot read %s\n", argv[2]); return 1; }
  HIP_OK(hipMemcpy(u, h, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
  if (!read_vec(argv[3], h, n)) { fprintf(stderr, "cannot read %s\n", argv[3]); return 1; }
  HIP_OK(hipMemcpy(x, h, (size_t)n * sizeof(double), hipMemcpyHostToDevice));

  double min_j = 0.0;
  MFH_OK(mfh_set_deformation(P, u, &min_j), P);
  MFH_OK(mfh_tangent_vmult(P, d.n_levels - 1, MFH_F64, x, y), P);
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(h, y, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
  if (!write_vec(argv[4], h, n)) { fprintf(stderr, "cannot write %s\n", argv[4]); return 1; }

  int iters = 0;
  double relres = 0.0;
  MFH_OK(mfh_cg_solve(P, x, z, 1e-8, 200, &iters, &relres), P);
  HIP_OK(hipMemcpy(h, z, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
  if (!write_vec(argv[5], h, n)) { fprintf(stderr, "cannot write %s\n", argv[5]); return 1; }
  printf("n_dofs %lld min_J %.6f cg_iters %d relres %.3e\n", n, min_j, iters, relres);

  MFH_OK(mfh_destroy(P), NULL);
  hipFree(z);
  hipFree(y);
  hipFree(x);
  hipFree(u);
  hipFree(ws);
  free(h);
  return 0;
}
