// Internal declarations shared by the kernels' translation units and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include "common.h"

namespace mlfft {

constexpr int kMaxGrid = 32;      // largest Nx, Ny handled by the in-register FFT codelets

// One array's share of a grouped 2-D FFT launch over W columns.
// Spatial layout (paper order of a column): in[w][iy][ix][m], m < b.
// Spectral layout: out[k][w][m] with k = ky*Px + kx.
// pad = 1: the Py x Px = 2Ny x 2Nx circulant grid of the MLFFT product (input
//          zero-padded, inverse output cropped to Ny x Nx);
// pad = 0: the Ny x Nx torus of the block-circulant preconditioner.
struct FftTask {
    const void* in;
    void* out;
    const void* addend;     // inverse only: optional, same layout as out
    double alpha;           // inverse only: out = alpha * F^{-1}(in) [+ beta * addend]
    double beta;
    int Nx, Ny, b, W;
    int cm;                 // basis functions per workgroup (m chunk)
    int rs;                 // row stride of the LDS tile in elements (>= Nx * cm)
    int nmc;                // number of m chunks
    int block_begin;        // first workgroup of this task in the grouped grid
    int pad;
    int colpad = 0;         // elements after each spatial column of in (forward) / out and addend (inverse):
                            // spatial columns start every Ny Nx b + colpad elements (the border unknowns of
                            // the full system follow the array's in every column); 0: back to back
    int out16 = 0;          // forward FP32, one-pass tile only: the spectrum is stored as bf16 (re, im) pairs
                            // (round to nearest even), 4 bytes per value, same layout
    int reserved = 0;       // fills the tail: a task's bytes are all defined (tables are cached by content)
};

// One array's share of a grouped per-frequency block product
// Y[k][w][m] = sum_n G[k][m][n] X[k][w][n]  (k < K, w < W, m, n < b).
struct GemmTask {
    const void* G;          // [K][b][b] complex (double2 / float2 / bf16 pairs)
    const void* X;          // [K][W][b]
    void* Y;                // [K][W][b]
    long gstride;           // elements between consecutive G[k] (b*b; 0 = one G shared by all k)
    int K, b, W;
    int mgroups;            // workgroups per frequency (row groups)
    int block_begin;
    int x16 = 0;            // bf16 product form 5 only: X holds bf16 (re, im) pairs instead of FP32 complex
};

// no padding bytes: the members add up to the size
static_assert(sizeof(FftTask) == 5 * 8 + 12 * 4, "FftTask must have no padding");
static_assert(sizeof(GemmTask) == 4 * 8 + 6 * 4, "GemmTask must have no padding");

enum Prec { P64 = 0, P32 = 1, PBF16 = 2 };

// launchers (return hipError_t of the launch)
hipError_t launch_fft_fwd(int prec, const FftTask* tasks_host, const FftTask* tasks_dev, int ntasks,
                          hipStream_t s);
hipError_t launch_fft_inv(int prec, const FftTask* tasks_host, const FftTask* tasks_dev, int ntasks,
                          hipStream_t s);
// fills cm / nmc / block_begin for a list of tasks of one direction (dir 0 forward,
// 1 inverse); returns the total grid size and the block size / dynamic LDS bytes the
// grouped launch needs
void plan_fft_tasks(int prec, FftTask* tasks, int ntasks, int dir, int* grid, int* block, size_t* lds);
// key of the launch a task joins: its tile kind (one-pass or half-height), its length
// class and its LDS tile size rounded up to a power of two
int fft_group_key(int prec, const FftTask& t, int dir);

// tuned FFT m-chunk (basis functions per workgroup) and tile kind per (prec, pad, dir,
// shape); cm <= 0 keeps the default rule, half < 0 the default tile
void fft_set_choice(int prec, int pad, int dir, int Nx, int Ny, int b, int cm, int half);
// the tuned m-chunk (0: default rule) and the tile kind in force (1: half-height)
void fft_get_choice(int prec, int pad, int dir, int Nx, int Ny, int b, int* cm, int* half);
bool fft_use_half(int prec, int pad, int dir, int Nx, int Ny, int b);
int fft_max_cm(int prec, int pad, int half, int Nx, int Ny, int b);

// tag 0: MLFFT spectra, 1: preconditioner (separate kernel symbols for profilers)
hipError_t launch_bgemm(int prec, const GemmTask* tasks_host, const GemmTask* tasks_dev, int ntasks, int tag,
                        hipStream_t s);
void plan_gemm_tasks(int prec, GemmTask* tasks, int ntasks, int tag, int* grid, int* bp_max);
// tuned launch shape of the MLFFT block product (waves per workgroup 4 or 8; columns per tile:
// FP64 16 or 32, FP32 / BF16 32 or 64; FP32 three-product form m3 = 1)
void gemm_set_shape(int prec, int bp, int waves, int nt, int m3);
// launch shape of the bf16 preconditioner product (waves 0: the default, one frequency per workgroup)
void gemm_set_pc_shape(int bp, int waves, int nt, int m3);
// workgroups a launch of the bf16 preconditioner's frequency kernel aims at (columns split to reach it)
void gemm_set_pc_wg_target(int n);
// whether the bf16 preconditioner product of arrays with these b (all of one padded b)
// reads its spectra in bf16 (form 5 moving pairs; every b even)
bool bf16_spectrum_ok(const int* b, int n);
void gemm_get_shape(int prec, int bp, int* waves, int* nt, int* m3);
int gemm_bp(int prec, int b);

// spectra / preconditioner setup (all FP64)
hipError_t launch_lag_dft_x(const double2* R, double2* T, int nlagy, int nlagx, int lagx0, int Px,
                            const double* wx, int bb, hipStream_t s);
hipError_t launch_lag_dft_y(const double2* T, double2* G, int nlagy, int lagy0, int Py, int Px,
                            const double* wy, int bb, hipStream_t s);
hipError_t launch_cast_c64_to_c32(const double2* a, float2* b, size_t n, hipStream_t s);
hipError_t launch_cast_c64_to_bf16(const double2* a, uint32_t* b, size_t n, hipStream_t s);
hipError_t launch_batched_inverse(double2* A, double2* Ainv, double* rcond, int* info, int nb, int b,
                                  hipStream_t s);
hipError_t launch_fill_identity_fallback(double2* Sinv, const double2* R00inv, const int* bad,
                                         int nb, int b, hipStream_t s);

}  // namespace mlfft

namespace mlfft {
hipError_t launch_nonfinite(const double* a, size_t n, int* flag, hipStream_t s);
// out = alpha * x + beta * y over n complex values (y may be NULL); in_prec / out_prec: P64 or P32
hipError_t launch_axpby(int in_prec, const void* x, const void* y, double alpha, double beta, int out_prec, void* out,
                        size_t n, hipStream_t s);
hipError_t launch_replicate(double2* dst, const double2* src, int nb, int bb, hipStream_t s);
}  // namespace mlfft
