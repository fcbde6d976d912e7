// Host-side state of the MLFFT library (contexts, arrays, workspaces).
#pragma once
#include <map>
#include <unordered_map>
#include <string>
#include <vector>

#include "internal.h"
#include "../../include/mlfft.h"

namespace mlfft {

// Incremented whenever any library buffer is allocated or freed: a captured
// graph holds raw device addresses and is valid only while this is unchanged.
extern unsigned long g_mem_epoch;

// The caller's device allocator (mlfft_create): every device buffer of the
// library comes from it and goes back to it.
struct Alloc {
    mlfft_alloc_fn fn = nullptr;
    mlfft_free_fn fr = nullptr;
    void* user = nullptr;
};

// A device buffer drawn from the context's allocator.  bind() names the
// allocator; ensure() grows the buffer (contents are not kept).
struct Buf {
    void* p = nullptr;
    size_t n = 0;
    const Alloc* al = nullptr;
    Buf() = default;
    explicit Buf(const Alloc* a) : al(a) {}
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    Buf(Buf&& o) noexcept : p(o.p), n(o.n), al(o.al) { o.p = nullptr; o.n = 0; }
    Buf& operator=(Buf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; al = o.al; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~Buf() { release(); }
    void bind(const Alloc* a) { al = a; }
    hipError_t ensure(size_t bytes);
    void release();
};

struct Array {
    int Nx = 0, Ny = 0, b = 0, Px = 0, Py = 0, K = 0;
    Buf G64, G32, G16;      // block spectra [K][b][b]: complex128, complex64, bf16 pairs
    Buf S64, S32, S16;      // Strang preconditioner inverse spectra [Nx*Ny][b][b]
    Buf K64, K32, K16;      // self-block inverse R_{0,0}^{-1}
    Buf R64;                // the unique blocks R_{p,q} as given, [p+Ny-1][q+Nx-1][m][n] (direct solver, P'_Z)
    Buf Z64, Z32;           // row preconditioner P'_Z: (T^[1]_0)^{-1}, (Nx b) x (Nx b) column-major (built on first use)
    double row_rcond = 0.0; // 1-norm reciprocal condition number of T^[1]_0 (0 until built)
    // border of the full matrix Z = [[Z_A, Z_B^T], [Z_B, Z_C]] (eq. Zblock), all column-major:
    // B (Nc x N) = Z_B, Bt (N x Nc) = Z_B^T, C (Nc x Nc) = Z_C, Ci = Z_C^{-1}, Kc = R_{0,0}^{-1}
    int Nc = 0;
    Buf B64, B32, Bt64, Bt32, C64, C32, Ci64, Ci32, Kc64, Kc32;
    size_t NA() const { return (size_t)Nx * Ny * b; }
    size_t Nt() const { return NA() + (size_t)Nc; }      // unknowns per column of the full system
    int pc_fallbacks = 0;
    double pc_min_rcond = 1.0;
    size_t bytes() const;
    void release();
    void bind(const Alloc* a) {
        for (Buf* b : {&G64, &G32, &G16, &S64, &S32, &S16, &K64, &K32, &K16, &R64, &Z64, &Z32, &B64, &B32, &Bt64,
                       &Bt32, &C64, &C32, &Ci64, &Ci32, &Kc64, &Kc32})
            b->bind(a);
    }
};

// y = alpha * Op(x) + beta * addend for one array (W columns)
struct MatvecItem {
    const Array* arr;
    int W;
    const void* x;
    void* y;
    const void* addend;
    double alpha;
    double beta;
};

}  // namespace mlfft

namespace mlfft {
// One profiled launch: HIP events recorded on the context's stream around it,
// with the algorithmic bytes and flops of that launch.
struct ProfRec {
    int kind;
    int prec;
    hipEvent_t a, b;
    double bytes, flops;
};
enum ProfKind { PK_FFT_FWD = 0, PK_GEMM, PK_FFT_INV, PK_PC_FFT_FWD, PK_PC_GEMM, PK_PC_FFT_INV, PK_ARNOLDI,
                PK_NET_FWD, PK_NET_BWD, PK_BORDER, PK_COUNT };
}  // namespace mlfft

struct mlfft_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    mlfft::Alloc alloc;            // the caller's device allocator
    std::string err;
    std::map<int, mlfft::Array> arrays;
    mlfft::Buf spec_a, spec_b;     // spectral workspaces of the matvec / preconditioner
    // Device copies of grouped-launch task tables, by content: offsets into the
    // device arena task_dev, filled by asynchronous copies from the pinned
    // staging arena task_host (same layout); task_used bytes of task_cap in use.
    std::unordered_map<std::string, size_t> task_cache;
    mlfft::Buf task_dev;
    unsigned char* task_host = nullptr;
    size_t task_cap = 0, task_used = 0;
    mlfft::Buf solve_ws;           // Krylov workspace (solve.cpp)
    mlfft::Buf solve_ws2;
    int* pinned = nullptr;         // pinned host buffer for per-column state read-back
    int pinned_n = 0;
    struct Net* net = nullptr;     // learned preconditioner (netapi.cpp)

    // Krylov steps captured as HIP graphs (solve option use_graph), keyed by the
    // step's launch configuration; all dropped when g_mem_epoch moves.
    std::map<std::string, hipGraphExec_t> graphs;
    std::map<std::string, int> graph_seen;
    unsigned long graph_epoch = 0;
    bool capturing = false;
    void graphs_release() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
        graph_seen.clear();
    }

    bool prof = false;
    std::vector<mlfft::ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used = 0;
    // start / stop a profiled launch (no-ops unless profiling is enabled)
    int prof_begin(int kind, int prec, double bytes, double flops);
    void prof_end(int rec);
    void prof_release();

    int* pinned_state(int n);
    bool net_ready() const;
    // z = learned correction of the block-circulant output y (W columns of array a)
    mlfft_status net_correct(const mlfft::Array* a, int W, const void* y, void* z, int prec, int* fallbacks);
    void net_release();
    int net_fallbacks_take();      // columns whose learned output was replaced since the last call

    mlfft_status fail(mlfft_status st, const char* fmt, ...);
    mlfft_status hip_fail(hipError_t e, const char* what);
    mlfft::Array* find(int id);
    mlfft_status upload_tasks(const void* host, size_t bytes, void** dev);
    mlfft_status gemm_grouped(int prec, std::vector<mlfft::GemmTask>& gm, int tag, const char* what);
    mlfft_status fft_grouped(int prec, std::vector<mlfft::FftTask>& tasks, bool inverse, const char* what);
    // ws_a, ws_b: spectral workspaces of ws_bytes each supplied by the caller (both NULL: the
    // context's own spec_a, spec_b, grown as needed)
    mlfft_status matvec_group(const std::vector<mlfft::MatvecItem>& items, int prec, void* ws_a = nullptr,
                              void* ws_b = nullptr, size_t ws_bytes = 0);
    mlfft_status precond_group(const std::vector<mlfft::MatvecItem>& items, int kind, int prec);
    // P'_Z of Sec. III-B: (T^[1]_0)^{-1} of array a, built once (dense.cpp)
    mlfft_status row_precond_setup(mlfft::Array& a);
    // border terms of y = alpha Z x + beta v for the arrays with a border (dense.cpp): runs after the
    // Z_A part has written alpha Z_A x_A + beta v_A into y_A
    mlfft_status border_matvec(const std::vector<mlfft::MatvecItem>& items, int prec);
    // border part of P_X^{-1}: z_C = Z_C^{-1} r_C
    mlfft_status border_precond(const std::vector<mlfft::MatvecItem>& items, int prec);
    void release_workspaces() {
        graphs_release();
        spec_a.release(); spec_b.release(); solve_ws.release(); solve_ws2.release();
        task_cache.clear();
        task_dev.release();
        if (task_host) (void)hipHostFree(task_host);
        task_host = nullptr;
        task_cap = task_used = 0;
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        pinned_n = 0;
        net_release();
        prof_release();
    }
};

typedef mlfft_ctx_s Ctx;

namespace mlfft {
// device address of the fixed scratch of mlfft_matvec_noalloc on `device` (the current device)
hipError_t scratch_init(int device);
}  // namespace mlfft

int prec_elem_bytes(int prec);
