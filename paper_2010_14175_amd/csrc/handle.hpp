// The opaque preconditioner handle behind afsai_precond.
#pragma once

#include <vector>

#include "sell.hpp"

struct afsai_precond_s {
    int device = -1;
    int32_t n = 0;
    int64_t nnz_g = 0;
    int32_t g_prec = AFSAI_F64;
    int32_t mmax = 1;
    // G (lower triangular) as CSR, for afsai_export
    int32_t *g_rp = nullptr, *g_ci = nullptr;
    void *g_val = nullptr;  // double* or float*
    // G and G^T in the SELL-64 layout used by afsai_apply and pcg_solve
    afsai::Sell sg, sgt;
    // per-row diagnostics (device)
    double *psi = nullptr;
    int32_t *steps = nullptr;
    int32_t *reason = nullptr;
    // workspace for apply (t) and PCG (r, z, p, q, t) and reductions
    double *work = nullptr;
    size_t work_elems = 0;
    afsai_setup_info info{};
    // batch of independent systems (afsai_setup_batched): first row of each system, nsys + 1
    // entries; empty for a single system
    std::vector<int32_t> seg_row0;
};

// The opaque prepared-matrix handle behind afsai_matrix: A's SELL-64 layout, converted once.
struct afsai_matrix_s {
    int device = -1;
    afsai_csr A{};  // the caller's CSR (n, nnz; its arrays are not read after the conversion)
    afsai::Sell S;
};

namespace afsai {
// A single-system solve as a task for the serving loop (solve.hip): begin enqueues the start
// on `stream`; advance never waits when block is false; finish waits and fills info.
struct PcgTask;
int pcg_task_begin(const afsai_csr &A, afsai_precond P, const double *b, double *x, double rtol, int32_t maxit,
                   hipStream_t stream, PcgTask **out);
int pcg_task_advance(PcgTask *t, bool block, bool *finished);
int pcg_task_finish(PcgTask *t, afsai_pcg_info *info);
void pcg_task_free(PcgTask *t);
}  // namespace afsai
