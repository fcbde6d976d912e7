// Launchers of the batched Krylov kernels (krylov.hip).
#pragma once
#include "internal.h"

namespace mlfft {

// Column descriptors of a (possibly multi-array) batch of vectors: column w
// starts at element off[w] (device array) and has N[w] entries (device array);
// a full vector holds S elements; maxN = max_w N[w].
struct Cols {
    const size_t* off;
    const int* N;
    int W;
    size_t S;
    size_t maxN;
    // Arnoldi chunking: column w owns chunks choff[w] .. choff[w+1]-1 (device,
    // W+1 entries, arnoldi_chunks(N[w]) each), nch chunks in all; part1 holds
    // the per-chunk partial sums coefficient-major, (4m+3) x nch doubles, and
    // hsum1 their per-column totals, W x (4m+3) doubles; gram the Gram matrix of
    // each column's basis, W x (m+1) x (m+1) complex doubles, needed with
    // orth == 2 (all device)
    const int* choff = nullptr;
    int nch = 0;
    int maxch = 0;              // largest number of chunks of one column
    double* part1 = nullptr;
    double* hsum1 = nullptr;
    double2* gram = nullptr;
};

// chunks of kArnChunk entries one column of N entries is cut into by k_arnoldi
int arnoldi_chunks(size_t N);

template<typename C> hipError_t k_colnorm(const void* x, const Cols& c, double* out, hipStream_t s);
template<typename C> hipError_t k_arnoldi(void* Vb, int j, const Cols& c, double2* H, int m, const int* state,
                                          int orth, hipStream_t s);
hipError_t k_givens(double2* H, double* cs, double2* sn, double2* g, int j, int m, int W, int* state,
                    const double* target, int* kcyc, int* iters, double* est, double* hist, int hist_len,
                    const double* scale, hipStream_t s);
template<typename C> hipError_t k_cycle_start(const void* r, void* v0, const Cols& c, double2* g, int m, int* state,
                                              const double* target, int* kcyc, double* est, hipStream_t s);
hipError_t k_lsq(const double2* H, const double2* g, double2* y, const int* kcyc, int m, int W, hipStream_t s);
// out_w (+)= sum_{i < kcyc[w]} y[w][i] B_i[w]; kmax >= every kcyc[w], 1 <= kmax <= m
template<typename C> hipError_t k_combine(const void* B, const Cols& c, const double2* y, const int* kcyc, int m,
                                          int kmax, void* out, int acc, hipStream_t s);
template<typename C> hipError_t k_add_cols(void* dst, const void* src, const Cols& c, hipStream_t s);
template<typename A, typename B> hipError_t k_scale_cols(const void* src, void* dst, const Cols& c, const double* sc,
                                                         int invert, hipStream_t s);
// x += sc[w] d in the columns with mask[w] set (mask NULL: all); assign != 0
// writes x = sc[w] d there and zero in the other columns instead (x is not read)
template<typename C> hipError_t k_axpy_cols(double2* x, const void* d, const Cols& c, const double* sc,
                                            const int* mask, int assign, hipStream_t s);

}  // namespace mlfft
