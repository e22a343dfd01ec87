// sf_spmv.hip -- the sparse matrix-vector products of Section 4.1 around the
// SF: a row-distributed matrix is split into a diagonal block A and an
// off-diagonal block B over the ghost vector lvec, and
//   y = M x:    SFBcast(x -> lvec) overlapped with y = A x, then y += B lvec;
//   y = M^T x:  y = A^T x, lvec = B^T x, then SFReduce SUM(lvec -> y).
// The CSR products are plain HIP kernels: G lanes of a wavefront per row
// (G a power of two near the mean row length), each lane striding over the
// row's entries, the lanes' partial sums combined by shuffles.
#include <algorithm>
#include <new>
#include <vector>

#include "sf_device.h"

struct sf_csr_s {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  std::vector<int64_t> h_rowptr;  // host copies (for the transpose)
  std::vector<int32_t> h_colidx;
  std::vector<double> h_values;
  int64_t *rowptr = nullptr;  // device
  int32_t *colidx = nullptr;
  double *values = nullptr;
  hipEvent_t ev = nullptr;  // the Bcast's completion, for the overlapped product
  int device = -1;
  int group = 1;  // lanes per row
};

namespace sfi {

template <int G>
__global__ __launch_bounds__(kBlock) void k_csr_spmv(const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ colidx,
                                                     const double *__restrict__ values, int64_t nrows,
                                                     const double *__restrict__ x, double *__restrict__ y,
                                                     int accumulate) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t row = gid / G;
  const int sub = (int)(gid % G);
  const bool ok = row < nrows;
  double s = 0.0;
  if (ok) {
    const int64_t k0 = rowptr[row], k1 = rowptr[row + 1];
    for (int64_t k = k0 + sub; k < k1; k += G) s += ld_stream(values + k) * x[ld_stream(colidx + k)];
  }
#pragma unroll
  for (int d = G / 2; d >= 1; d /= 2) s += __shfl_xor(s, d, G);
  if (ok && sub == 0) y[row] = accumulate ? y[row] + s : s;
}

static int pick_group(int64_t nrows, int64_t nnz) {
  const double mean = nrows > 0 ? (double)nnz / (double)nrows : 1.0;
  int g = 1;
  while (g < 64 && g < mean) g *= 2;
  return g;
}

static int csr_launch(const sf_csr_s *a, const double *x, double *y, int accumulate, hipStream_t st) {
  if (a->nrows == 0) return SF_OK;
  const int64_t threads = a->nrows * a->group;
  const unsigned g = (unsigned)((threads + kBlock - 1) / kBlock);
#define SF_CSR(G)                                                                                                 \
  case G:                                                                                                         \
    hipLaunchKernelGGL((k_csr_spmv<G>), dim3(g), dim3(kBlock), 0, st, a->rowptr, a->colidx, a->values, a->nrows, x, \
                       y, accumulate);                                                                            \
    break
  switch (a->group) {
    SF_CSR(1);
    SF_CSR(2);
    SF_CSR(4);
    SF_CSR(8);
    SF_CSR(16);
    SF_CSR(32);
    default: SF_CSR(64);
  }
#undef SF_CSR
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SF_OK : set_hip_error(e);
}

static void csr_free(sf_csr_s *a) {
  if (a->rowptr) (void)hipFree(a->rowptr);
  if (a->colidx) (void)hipFree(a->colidx);
  if (a->values) (void)hipFree(a->values);
  if (a->ev) (void)hipEventDestroy(a->ev);
  delete a;
}

static int csr_upload(sf_csr_s *a) {
  hipError_t e = hipGetDevice(&a->device);
  if (e == hipSuccess) e = hipMalloc(&a->rowptr, (size_t)(a->nrows + 1) * 8);
  if (e == hipSuccess) e = hipMalloc(&a->colidx, (size_t)std::max<int64_t>(a->nnz, 1) * 4);
  if (e == hipSuccess) e = hipMalloc(&a->values, (size_t)std::max<int64_t>(a->nnz, 1) * 8);
  if (e == hipSuccess) e = hipMemcpy(a->rowptr, a->h_rowptr.data(), (size_t)(a->nrows + 1) * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && a->nnz)
    e = hipMemcpy(a->colidx, a->h_colidx.data(), (size_t)a->nnz * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && a->nnz)
    e = hipMemcpy(a->values, a->h_values.data(), (size_t)a->nnz * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&a->ev, hipEventDisableTiming);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? SF_ERR_OOM : set_hip_error(e);
  a->group = pick_group(a->nrows, a->nnz);
  return SF_OK;
}

}  // namespace sfi

using namespace sfi;

extern "C" int sf_csr_create(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
                             const double *values, sf_csr_t *out) {
  if (!out) return SF_ERR_ARG;
  *out = nullptr;
  if (nrows < 0 || ncols < 0 || nrows > INT32_MAX || ncols > INT32_MAX || !rowptr) return SF_ERR_ARG;
  if (rowptr[0] != 0) return SF_ERR_ARG;
  for (int64_t i = 0; i < nrows; i++)
    if (rowptr[i + 1] < rowptr[i]) return SF_ERR_ARG;
  const int64_t nnz = rowptr[nrows];
  if (nnz > 0 && (!colidx || !values)) return SF_ERR_ARG;
  for (int64_t k = 0; k < nnz; k++)
    if (colidx[k] < 0 || colidx[k] >= ncols) return SF_ERR_ARG;
  auto *a = new (std::nothrow) sf_csr_s();
  if (!a) return SF_ERR_OOM;
  try {
    a->nrows = nrows;
    a->ncols = ncols;
    a->nnz = nnz;
    a->h_rowptr.assign(rowptr, rowptr + nrows + 1);
    a->h_colidx.assign(colidx, colidx + nnz);
    a->h_values.assign(values, values + nnz);
  } catch (const std::bad_alloc &) {
    delete a;
    return SF_ERR_OOM;
  }
  int rc = csr_upload(a);
  if (rc) {
    csr_free(a);
    return rc;
  }
  *out = a;
  return SF_OK;
}

extern "C" int sf_csr_transpose(sf_csr_t a, sf_csr_t *out) {
  if (!a || !out) return SF_ERR_ARG;
  *out = nullptr;
  // counting sort of the entries by column; inside a column, by row
  std::vector<int64_t> rp((size_t)a->ncols + 1, 0);
  std::vector<int32_t> ci((size_t)a->nnz);
  std::vector<double> va((size_t)a->nnz);
  for (int64_t k = 0; k < a->nnz; k++) rp[(size_t)a->h_colidx[k] + 1]++;
  for (int64_t j = 0; j < a->ncols; j++) rp[j + 1] += rp[j];
  std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
  for (int64_t i = 0; i < a->nrows; i++)
    for (int64_t k = a->h_rowptr[i]; k < a->h_rowptr[i + 1]; k++) {
      const int64_t at = fill[a->h_colidx[k]]++;
      ci[at] = (int32_t)i;
      va[at] = a->h_values[k];
    }
  return sf_csr_create(a->ncols, a->nrows, rp.data(), ci.data(), va.data(), out);
}

extern "C" int sf_csr_spmv(sf_csr_t a, const double *x, double *y, int32_t accumulate, hipStream_t stream) {
  if (!a || (a->nrows > 0 && (!y || (a->ncols > 0 && !x)))) return SF_ERR_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != a->device) return SF_ERR_ARG;
  return csr_launch(a, x, y, accumulate ? 1 : 0, stream);
}

extern "C" int sf_csr_destroy(sf_csr_t *a) {
  if (!a) return SF_ERR_ARG;
  if (*a) csr_free(*a);
  *a = nullptr;
  return SF_OK;
}

extern "C" int sf_spmv(sf_t sf, sf_csr_t A, sf_csr_t B, const double *x, double *lvec, double *y, hipStream_t stream,
                       hipStream_t comm_stream) {
  if (!sf || !A || !B) return SF_ERR_ARG;
  if (A->nrows != B->nrows || A->ncols != sf->nroots || B->ncols != sf->leafspace) return SF_ERR_ARG;
  const sf_unit u{SF_F64, 1};
  // the ghost values travel on comm_stream while the local product runs
  int rc = sf_bcast_begin(sf, u, x, lvec, SF_REPLACE, comm_stream);
  if (rc) return rc;
  hipError_t e = hipEventRecord(A->ev, comm_stream);
  if (e != hipSuccess) return set_hip_error(e);
  rc = sf_csr_spmv(A, x, y, 0, stream);
  if (rc) return rc;
  e = hipStreamWaitEvent(stream, A->ev, 0);
  if (e != hipSuccess) return set_hip_error(e);
  rc = sf_bcast_end(sf, u, x, lvec, SF_REPLACE, comm_stream);
  if (rc) return rc;
  return sf_csr_spmv(B, lvec, y, 1, stream);
}

extern "C" int sf_spmv_transpose(sf_t sf, sf_csr_t At, sf_csr_t Bt, const double *x, double *lvec, double *y,
                                 hipStream_t stream) {
  if (!sf || !At || !Bt) return SF_ERR_ARG;
  if (At->ncols != Bt->ncols || At->nrows != sf->nroots || Bt->nrows != sf->leafspace) return SF_ERR_ARG;
  const sf_unit u{SF_F64, 1};
  int rc = sf_csr_spmv(At, x, y, 0, stream);
  if (!rc) rc = sf_csr_spmv(Bt, x, lvec, 0, stream);
  if (!rc) rc = sf_reduce_begin(sf, u, lvec, y, SF_SUM, stream);
  if (!rc) rc = sf_reduce_end(sf, u, lvec, y, SF_SUM, stream);
  return rc;
}
