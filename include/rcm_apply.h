/*
 * rcm_apply.h -- applying an ordering on the GPU: the permuted matrix
 * B = P A P^T and a sparse matrix-vector product, as a C ABI.
 *
 * The paper motivates the ordering by where it puts the nonzeros: a small
 * bandwidth clusters them near the diagonal, which improves data locality in
 * iterative methods (Section I; Fig. 1 shows a conjugate-gradient solve on a
 * matrix whose bandwidth falls from 1,226,000 to 795).  These calls build
 * the reordered matrix and run the kernel such a solver spends its time in,
 * so that the locality gained can be measured.
 *
 * Conventions (as in rcm.h): CSR arrays are DEVICE pointers owned by the
 * caller (int32 rowptr[n+1], int32 colidx[nnz], nnz < 2^31, no duplicate
 * entries in a row); values, when given, are float64[nnz] in the same order
 * as colidx; stream is a hipStream_t passed as void* (NULL = default
 * stream); work is enqueued on it and the calls return once it has been
 * enqueued (no host synchronisation).  Errors are returned as rcm_status.
 */
#ifndef RCM_APPLY_H_
#define RCM_APPLY_H_

#include <stddef.h>
#include <stdint.h>

#include "rcm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Workspace bytes rcm_permute needs for n rows, nnz entries, with or without
 * values.  Host arithmetic. */
size_t rcm_permute_workspace_bytes(int32_t n, int64_t nnz, int32_t with_values);

/* B = P A P^T for the ordering perm (new -> old) and its inverse iperm
 * (old -> new), as rcm_order_ex returns them: row k of B is row perm[k] of
 * A with every column j renamed iperm[j], its entries sorted by column.
 * rowptr_out int32[n+1] and colidx_out int32[nnz] (and vals_out float64[nnz]
 * when vals is given) are device outputs, disjoint from the inputs.
 * workspace: device, at least rcm_permute_workspace_bytes.
 * Errors: RCM_ERR_INVALID_ARGUMENT (n < 0, nnz < 0, NULL pointer with n > 0,
 * vals without vals_out), RCM_ERR_WORKSPACE_TOO_SMALL, RCM_ERR_HIP.
 * The inputs are not checked again: perm/iperm must be a permutation pair
 * and the CSR valid (what rcm_order_ex accepted). */
rcm_status rcm_permute(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                       const double* vals, const int32_t* perm, const int32_t* iperm,
                       int32_t* rowptr_out, int32_t* colidx_out, double* vals_out,
                       void* workspace, size_t workspace_bytes, void* stream);

/* y = A x in float64 for a CSR matrix (vals NULL: every stored entry is 1).
 * x, y: device float64[n], disjoint.  Each row is summed in column order of
 * its storage by a group of lanes, then reduced across the group (the
 * summation order differs from a sequential loop by rounding only).
 * Errors: RCM_ERR_INVALID_ARGUMENT, RCM_ERR_HIP. */
rcm_status rcm_spmv(int32_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                    const double* x, double* y, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RCM_APPLY_H_ */
