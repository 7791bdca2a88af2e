/* A plain C caller of the library's C ABI (test driver).
 *
 * Reads a problem from argv[1] (binary, native endianness):
 *   int32 dim, int64 n_vert, double vert[n_vert*dim], int64 n_elem,
 *   int32 elem[n_elem*(dim+1)], int32 has_canon, [int32 canon[n_vert]],
 *   int32 p, int32 flux, double gamma, int64 K, double u[K], double dt, int32 m
 * (a periodic mesh: no boundary faces), creates a context, computes R(u) and
 * one FP64 tangent PCEXP step from u with dt and m, and writes
 *   double R[K], double u_next[K], int32 m_eff1, int32 m_eff2
 * to argv[2].  Device memory comes from the HIP runtime; every library call's
 * status is checked and a failure prints pcexp_last_error and exits 1. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "pcexp.h"

#define READ(ptr, n)                                                     \
  do {                                                                   \
    if (fread((ptr), sizeof(*(ptr)), (size_t)(n), f) != (size_t)(n)) {  \
      fprintf(stderr, "short read\n");                                   \
      return 1;                                                          \
    }                                                                    \
  } while (0)

#define HIPCHECK(x)                                                      \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      fprintf(stderr, "HIP error %d at %s\n", (int)e_, #x);              \
      return 1;                                                          \
    }                                                                    \
  } while (0)

static int check(pcexp_status s, const pcexp_ctx* c, const char* what) {
  if (s != PCEXP_OK) {
    fprintf(stderr, "%s failed (%d): %s\n", what, (int)s, c ? pcexp_last_error(c) : "");
    return 1;
  }
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 1;
  int32_t dim, has_canon, p, flux, m;
  int64_t n_vert, n_elem, K;
  double gamma, dt;
  READ(&dim, 1);
  READ(&n_vert, 1);
  double* vert = (double*)malloc(sizeof(double) * n_vert * dim);
  READ(vert, n_vert * dim);
  READ(&n_elem, 1);
  int32_t* elem = (int32_t*)malloc(sizeof(int32_t) * n_elem * (dim + 1));
  READ(elem, n_elem * (dim + 1));
  READ(&has_canon, 1);
  int32_t* canon = NULL;
  if (has_canon) {
    canon = (int32_t*)malloc(sizeof(int32_t) * n_vert);
    READ(canon, n_vert);
  }
  READ(&p, 1);
  READ(&flux, 1);
  READ(&gamma, 1);
  READ(&K, 1);
  double* u = (double*)malloc(sizeof(double) * K);
  READ(u, K);
  READ(&dt, 1);
  READ(&m, 1);
  fclose(f);

  pcexp_mesh_desc mesh = {dim, n_vert, vert, n_elem, elem, canon, 0, NULL, NULL};
  pcexp_disc_desc disc = {p, flux, gamma, {1.0, 0.0, 0.0, 0.0, 1.0}};
  pcexp_ctx* ctx = NULL;
  if (check(pcexp_create(&mesh, &disc, NULL, &ctx), NULL, "pcexp_create")) return 1;
  int64_t sizes[8];
  if (check(pcexp_sizes(ctx, sizes), ctx, "pcexp_sizes")) return 1;
  if (sizes[0] != K) {
    fprintf(stderr, "size mismatch: library K %lld, input K %lld\n", (long long)sizes[0], (long long)K);
    return 1;
  }

  double *du, *dR;
  HIPCHECK(hipMalloc((void**)&du, sizeof(double) * K));
  HIPCHECK(hipMalloc((void**)&dR, sizeof(double) * K));
  HIPCHECK(hipMemcpy(du, u, sizeof(double) * K, hipMemcpyHostToDevice));
  if (check(pcexp_residual(ctx, du, dR, NULL), ctx, "pcexp_residual")) return 1;

  const size_t wsb = pcexp_workspace_bytes(ctx, m, 1, PCEXP_PREC_F64, PCEXP_JVP_TANGENT);
  void* ws = NULL;
  HIPCHECK(hipMalloc(&ws, wsb));
  pcexp_step_info info;
  if (check(pcexp_step(ctx, du, dt, 0.0, m, PCEXP_SCHEME_PCEXP, PCEXP_PREC_F64, PCEXP_JVP_TANGENT, ws, wsb, &info,
                       NULL),
            ctx, "pcexp_step"))
    return 1;
  HIPCHECK(hipDeviceSynchronize());

  double* R = (double*)malloc(sizeof(double) * K);
  HIPCHECK(hipMemcpy(R, dR, sizeof(double) * K, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(u, du, sizeof(double) * K, hipMemcpyDeviceToHost));
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 1;
  fwrite(R, sizeof(double), (size_t)K, o);
  fwrite(u, sizeof(double), (size_t)K, o);
  fwrite(&info.k1.m_eff, sizeof(int32_t), 1, o);
  fwrite(&info.k2.m_eff, sizeof(int32_t), 1, o);
  fclose(o);

  hipFree(ws);
  hipFree(dR);
  hipFree(du);
  pcexp_destroy(ctx);
  free(R);
  free(u);
  free(canon);
  free(elem);
  free(vert);
  printf("ok K=%lld m_eff=%d,%d\n", (long long)K, info.k1.m_eff, info.k2.m_eff);
  return 0;
}
