// C ABI of the MLFFT library: contexts, arrays (spectra and preconditioner
// setup), the MLFFT matvec and the preconditioner apply.  The Krylov solver
// driver lives in solve.cpp.
#include "lib.h"
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

using namespace mlfft;

static thread_local std::string g_create_error;

mlfft_status Ctx::fail(mlfft_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return st;
}

mlfft_status Ctx::hip_fail(hipError_t e, const char* what) {
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return fail(MLFFT_E_NOMEM, "%s: out of device memory", what);
    return fail(MLFFT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

unsigned long mlfft::g_mem_epoch = 1;

hipError_t Buf::ensure(size_t bytes) {
    if (n >= bytes && p) return hipSuccess;
    release();
    if (bytes == 0) return hipSuccess;
    if (!al || !al->fn) return hipErrorInvalidValue;     // a buffer never bound to an allocator
    ++g_mem_epoch;
    p = al->fn(bytes, al->user);
    if (!p) { n = 0; return hipErrorOutOfMemory; }
    n = bytes;
    return hipSuccess;
}

void Buf::release() {
    if (p) {
        ++g_mem_epoch;
        al->fr(p, al->user);
    }
    p = nullptr;
    n = 0;
}

int Ctx::prof_begin(int kind, int prec, double bytes, double flops) {
    if (!prof || capturing) return -1;
    while (prof_pool.size() < prof_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        prof_pool.push_back(e);
    }
    ProfRec r{kind, prec, prof_pool[prof_used], prof_pool[prof_used + 1], bytes, flops};
    prof_used += 2;
    (void)hipEventRecord(r.a, stream);
    prof_recs.push_back(r);
    return (int)prof_recs.size() - 1;
}

void Ctx::prof_end(int rec) {
    if (rec < 0) return;
    (void)hipEventRecord(prof_recs[rec].b, stream);
}

void Ctx::prof_release() {
    for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
    prof_pool.clear();
    prof_recs.clear();
    prof_used = 0;
}

int* Ctx::pinned_state(int n) {
    if (n > pinned_n) {
        if (pinned) (void)hipHostFree(pinned);
        ++g_mem_epoch;
        pinned = nullptr;
        pinned_n = 0;
        if (hipHostMalloc((void**)&pinned, (size_t)n * sizeof(int), hipHostMallocDefault) != hipSuccess) return nullptr;
        pinned_n = n;
    }
    return pinned;
}

Array* Ctx::find(int id) {
    auto it = arrays.find(id);
    return it == arrays.end() ? nullptr : &it->second;
}

size_t Array::bytes() const {
    size_t t = 0;
    for (const Buf* x : {&G64, &G32, &G16, &S64, &S32, &S16, &K64, &K32, &K16, &R64, &Z64, &Z32, &B64, &B32, &Bt64,
                         &Bt32, &C64, &C32, &Ci64, &Ci32, &Kc64, &Kc32})
        t += x->n;
    return t;
}

void Array::release() {
    G64.release(); G32.release(); G16.release();
    S64.release(); S32.release(); S16.release();
    K64.release(); K32.release(); K16.release();
    R64.release(); Z64.release(); Z32.release();
    for (Buf* x : {&B64, &B32, &Bt64, &Bt32, &C64, &C32, &Ci64, &Ci32, &Kc64, &Kc32}) x->release();
    row_rcond = 0.0;
    Nc = 0;
}

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return c->hip_fail(e_, what);  \
    } while (0)

#define STCHK(call)                                          \
    do {                                                     \
        mlfft_status s_ = (call);                            \
        if (s_ < 0) return s_;                               \
    } while (0)

int prec_elem_bytes(int prec) { return prec == P64 ? 16 : 8; }

// ------------------------------------------------------------------ matvec core

mlfft_status Ctx::upload_tasks(const void* host, size_t bytes, void** dev) {
    // Task tables are small and repeated solves reuse the same tables: each
    // distinct table is kept resident in a device arena.  A new one is copied
    // into the pinned staging arena and from there to the device with an
    // asynchronous copy on the stream, ordered before the launch that reads it,
    // so the stream does not drain.  A staging slot is written once per arena
    // cycle; starting a new cycle drains the stream first.
    Ctx* c = this;
    std::string key((const char*)host, bytes);
    auto it = task_cache.find(key);
    if (it != task_cache.end()) {
        *dev = (char*)task_dev.p + it->second;
        return MLFFT_OK;
    }
    // a graph capture replays only launches whose tables are already resident
    if (capturing) return fail(MLFFT_E_STATE, "task table not resident during graph capture");
    const size_t need = (bytes + 255) / 256 * 256;
    if (!task_host || task_used + need > task_cap) {
        HIPCHK(hipStreamSynchronize(stream), "task arena");
        task_cache.clear();
        task_used = 0;
        ++g_mem_epoch;                  // graphs may hold addresses of the old tables
        if (need > task_cap) {
            const size_t cap = std::max<size_t>(need, std::max<size_t>(8u << 20, 2 * task_cap));
            if (task_host) (void)hipHostFree(task_host);
            task_host = nullptr;
            task_cap = 0;
            HIPCHK(task_dev.ensure(cap), "task arena");
            HIPCHK(hipHostMalloc((void**)&task_host, cap, hipHostMallocDefault), "task arena");
            task_cap = cap;
        }
    }
    std::memcpy(task_host + task_used, host, bytes);
    HIPCHK(hipMemcpyAsync((char*)task_dev.p + task_used, task_host + task_used, bytes, hipMemcpyHostToDevice, stream),
           "task table upload");
    task_cache.emplace(std::move(key), task_used);
    *dev = (char*)task_dev.p + task_used;
    task_used += need;
    return MLFFT_OK;
}

// Block products of a group of arrays.  The kernels are instantiated for a
// padded reduction length BP and run every task of a launch at the largest
// one, so tasks are launched in groups of equal padded b: a small-b array is
// never padded to the b of a larger one.
mlfft_status Ctx::gemm_grouped(int prec, std::vector<GemmTask>& gm, int tag, const char* what) {
    Ctx* c = this;
    std::map<int, std::vector<GemmTask>> groups;
    for (const GemmTask& g : gm) groups[gemm_bp(prec, g.b)].push_back(g);
    for (auto& kv : groups) {
        std::vector<GemmTask>& sub = kv.second;
        const int n = (int)sub.size();
        int grid, bpm;
        plan_gemm_tasks(prec, sub.data(), n, tag, &grid, &bpm);
        void* d = nullptr;
        if (n > 1) {
            mlfft_status st = upload_tasks(sub.data(), sizeof(GemmTask) * n, &d);
            if (st != MLFFT_OK) return st;
        }
        HIPCHK(launch_bgemm(prec, sub.data(), (const GemmTask*)d, n, tag, stream), what);
    }
    return MLFFT_OK;
}

// 2-D FFTs of a group of arrays, one launch per (length class, LDS tile size):
// a grouped launch runs the kernel of its largest length class and reserves
// its largest tile for every workgroup, which would cost small arrays their
// occupancy.
mlfft_status Ctx::fft_grouped(int prec, std::vector<FftTask>& tasks, bool inverse, const char* what) {
    Ctx* c = this;
    // the transforms of the bf16-product forms are FP32 (and tuned as such)
    if (prec == PBF16) prec = P32;
    std::map<int, std::vector<FftTask>> groups;
    for (const FftTask& t : tasks) groups[fft_group_key(prec, t, inverse ? 1 : 0)].push_back(t);
    for (auto& kv : groups) {
        std::vector<FftTask>& sub = kv.second;
        const int n = (int)sub.size();
        int grid, block;
        size_t lds;
        plan_fft_tasks(prec, sub.data(), n, inverse ? 1 : 0, &grid, &block, &lds);
        void* d = nullptr;
        if (n > 1) {
            mlfft_status st = upload_tasks(sub.data(), sizeof(FftTask) * n, &d);
            if (st != MLFFT_OK) return st;
        }
        HIPCHK(inverse ? launch_fft_inv(prec, sub.data(), (const FftTask*)d, n, stream)
                       : launch_fft_fwd(prec, sub.data(), (const FftTask*)d, n, stream), what);
    }
    return MLFFT_OK;
}

// y = alpha * Z x + beta * addend over a group of arrays (one grouped launch per phase)
mlfft_status Ctx::matvec_group(const std::vector<MatvecItem>& items, int prec, void* ws_a, void* ws_b,
                                size_t ws_bytes) {
    Ctx* c = this;
    const int nt = (int)items.size();
    if (nt == 0) return MLFFT_OK;
    const int eb = prec_elem_bytes(prec);
    // spectral workspaces
    size_t need = 0;
    std::vector<size_t> off(nt);
    for (int i = 0; i < nt; ++i) {
        const Array* a = items[i].arr;
        off[i] = need;
        need += (size_t)a->K * a->b * items[i].W * eb;
        need = (need + 255) / 256 * 256;
    }
    char* sa;
    char* sb;
    if (ws_a || ws_b) {
        if (!ws_a || !ws_b || need > ws_bytes)
            return fail(MLFFT_E_ARG, "spectral workspace of %zu bytes needed, %zu supplied", need, ws_bytes);
        sa = (char*)ws_a;
        sb = (char*)ws_b;
    } else {
        HIPCHK(spec_a.ensure(need), "spectral workspace");
        HIPCHK(spec_b.ensure(need), "spectral workspace");
        sa = (char*)spec_a.p;
        sb = (char*)spec_b.p;
    }
    std::vector<FftTask> fw(nt), iv(nt);
    std::vector<GemmTask> gm(nt);
    for (int i = 0; i < nt; ++i) {
        const MatvecItem& it = items[i];
        const Array* a = it.arr;
        FftTask t{};
        t.in = it.x; t.out = sa + off[i]; t.addend = nullptr; t.alpha = 1.0; t.beta = 0.0;
        t.Nx = a->Nx; t.Ny = a->Ny; t.b = a->b; t.W = it.W; t.pad = 1; t.colpad = a->Nc;
        fw[i] = t;
        GemmTask g{};
        g.G = prec == P64 ? a->G64.p : prec == P32 ? a->G32.p : a->G16.p;
        g.X = sa + off[i]; g.Y = sb + off[i];
        g.K = a->K; g.b = a->b; g.W = it.W; g.gstride = (long)a->b * a->b;
        gm[i] = g;
        FftTask u{};
        u.in = sb + off[i]; u.out = it.y; u.addend = it.addend;
        u.alpha = it.alpha / (double)a->K; u.beta = it.beta;
        u.Nx = a->Nx; u.Ny = a->Ny; u.b = a->b; u.W = it.W; u.pad = 1; u.colpad = a->Nc;
        iv[i] = u;
    }
    // algorithmic bytes / flops of the three launches (s: bytes per complex of the data, sg: of the spectra)
    double bf = 0, bg = 0, bi = 0, fl = 0;
    const double s = eb, sg = prec == P64 ? 16 : prec == P32 ? 8 : 4;
    for (int i = 0; i < nt; ++i) {
        const Array* a = items[i].arr;
        const double N = (double)a->Nx * a->Ny * a->b * items[i].W, KB = (double)a->K * a->b * items[i].W;
        bf += s * (N + KB);
        bg += s * 2 * KB + sg * (double)a->K * a->b * a->b;
        bi += s * (KB + N + (items[i].addend ? N : 0));
        fl += 8.0 * a->K * (double)a->b * a->b * items[i].W;
    }
    int pr = prof_begin(PK_FFT_FWD, prec, bf, 0);
    STCHK(fft_grouped(prec, fw, false, "forward MLFFT launch"));
    prof_end(pr);
    pr = prof_begin(PK_GEMM, prec, bg, fl);
    STCHK(gemm_grouped(prec, gm, 0, "block product launch"));
    prof_end(pr);
    pr = prof_begin(PK_FFT_INV, prec, bi, 0);
    STCHK(fft_grouped(prec, iv, true, "inverse MLFFT launch"));
    prof_end(pr);
    return border_matvec(items, prec);
}

// z = alpha * P^{-1} r (+ beta * addend) with the block-circulant or self-block preconditioner
mlfft_status Ctx::precond_group(const std::vector<MatvecItem>& items, int kind, int prec) {
    Ctx* c = this;
    const int nt = (int)items.size();
    if (nt == 0) return MLFFT_OK;
    const int eb = prec_elem_bytes(prec);
    if (kind == 4) {
        // row preconditioner P'_Z: every row of cells of every column is one vector of
        // length Nx b, so the apply is one dense product (T^[1]_0)^{-1} [n x (Ny W)]
        // (batched over the columns when border unknowns sit between them)
        for (const MatvecItem& it : items) {
            Array* a = const_cast<Array*>(it.arr);
            if (it.addend || it.alpha != 1.0) return fail(MLFFT_E_ARG, "row preconditioner apply has no epilogue");
            STCHK(row_precond_setup(*a));
            const int n = a->Nx * a->b;
            const int p = prec == P64 ? 0 : 1;
            const double bytes = (double)eb * 2 * n * a->Ny * it.W + (p ? 8.0 : 16.0) * n * n;
            const double flops = 8.0 * n * (double)n * a->Ny * it.W;
            const int pr = prof_begin(PK_PC_GEMM, prec, bytes, flops);
            const void* Zi = p ? a->Z32.p : a->Z64.p;
            if (a->Nc == 0)
                HIPCHK(dense_gemm(p, n, a->Ny * it.W, n, make_double2(1.0, 0.0), Zi, n, 0, it.x, n, 0,
                                  make_double2(0.0, 0.0), it.y, n, 0, 1, stream), "row preconditioner apply");
            else
                HIPCHK(dense_gemm(p, n, a->Ny, n, make_double2(1.0, 0.0), Zi, n, 0, it.x, n, (long)a->Nt(),
                                  make_double2(0.0, 0.0), it.y, n, (long)a->Nt(), it.W, stream),
                       "row preconditioner apply");
            prof_end(pr);
        }
        return border_precond(items, prec);
    }
    if (kind == 2) {
        // self block: one b x b product per cell.  Arrays without a border run the block
        // product with the whole vector as one frequency; with border unknowns between the
        // columns it is a dense product R_{0,0}^{-1} [b x (Nx Ny)] batched over the columns.
        std::vector<GemmTask> gm;
        for (const MatvecItem& it : items) {
            const Array* a = it.arr;
            if (it.addend || it.alpha != 1.0) return fail(MLFFT_E_ARG, "self-block apply has no epilogue");
            if (a->Nc > 0) {
                const int p = prec == P64 ? 0 : 1;
                const long ld = (long)a->Nt();
                HIPCHK(dense_gemm(p, a->b, a->Nx * a->Ny, a->b, make_double2(1.0, 0.0), p ? a->Kc32.p : a->Kc64.p, a->b,
                                  0, it.x, a->b, ld, make_double2(0.0, 0.0), it.y, a->b, ld, it.W, stream),
                       "self-block apply");
                continue;
            }
            GemmTask g{};
            g.G = prec == P64 ? a->K64.p : prec == P32 ? a->K32.p : a->K16.p;
            g.X = it.x; g.Y = it.y; g.K = it.W; g.b = a->b; g.W = a->Nx * a->Ny; g.gstride = 0;
            gm.push_back(g);
        }
        if (!gm.empty()) STCHK(gemm_grouped(prec, gm, 1, "self-block apply launch"));
        return border_precond(items, prec);
    }
    size_t need = 0;
    std::vector<size_t> off(nt);
    for (int i = 0; i < nt; ++i) {
        const Array* a = items[i].arr;
        off[i] = need;
        need += (size_t)a->Nx * a->Ny * a->b * items[i].W * eb;
        need = (need + 255) / 256 * 256;
    }
    HIPCHK(spec_a.ensure(need), "preconditioner workspace");
    HIPCHK(spec_b.ensure(need), "preconditioner workspace");
    // bf16 products that read bf16 spectra (decided per padded b, the unit of a product
    // launch): the forward transform then stores its spectrum in bf16 pairs, which halves
    // its writes and the product's reads, with the same rounding the product would apply
    std::map<int, bool> spec16;
    if (prec == PBF16) {
        std::map<int, std::vector<int>> bs;
        for (const MatvecItem& it : items) bs[gemm_bp(PBF16, it.arr->b)].push_back(it.arr->b);
        for (auto& kv : bs) spec16[kv.first] = bf16_spectrum_ok(kv.second.data(), (int)kv.second.size());
    }
    std::vector<FftTask> fw(nt), iv(nt);
    std::vector<GemmTask> gm(nt);
    std::vector<int> x16(nt, 0);
    for (int i = 0; i < nt; ++i) {
        const MatvecItem& it = items[i];
        const Array* a = it.arr;
        x16[i] = prec == PBF16 && spec16[gemm_bp(PBF16, a->b)] ? 1 : 0;
        FftTask t{};
        t.in = it.x; t.out = (char*)spec_a.p + off[i]; t.alpha = 1.0;
        t.Nx = a->Nx; t.Ny = a->Ny; t.b = a->b; t.W = it.W; t.pad = 0; t.colpad = a->Nc;
        t.out16 = x16[i];
        fw[i] = t;
        GemmTask g{};
        g.G = prec == P64 ? a->S64.p : prec == P32 ? a->S32.p : a->S16.p;
        g.X = (char*)spec_a.p + off[i]; g.Y = (char*)spec_b.p + off[i];
        g.K = a->Nx * a->Ny; g.b = a->b; g.W = it.W; g.gstride = (long)a->b * a->b;
        g.x16 = x16[i];
        gm[i] = g;
        FftTask u{};
        u.in = (char*)spec_b.p + off[i]; u.out = it.y; u.addend = it.addend;
        u.alpha = it.alpha / (double)(a->Nx * a->Ny); u.beta = it.beta;
        u.Nx = a->Nx; u.Ny = a->Ny; u.b = a->b; u.W = it.W; u.pad = 0; u.colpad = a->Nc;
        iv[i] = u;
    }
    double bf = 0, bfw = 0, bg = 0, fl = 0;
    const double s = eb, sg = prec == P64 ? 16 : prec == P32 ? 8 : 4;
    for (int i = 0; i < nt; ++i) {
        const Array* a = items[i].arr;
        const double N = (double)a->Nx * a->Ny * a->b * items[i].W;
        const double sx = x16[i] ? 4 : s;       // bytes per value of the forward spectrum
        bf += s * 2 * N;
        bfw += (s + sx) * N;
        bg += (sx + s) * N + sg * (double)a->Nx * a->Ny * a->b * a->b;
        fl += 8.0 * a->Nx * a->Ny * (double)a->b * a->b * items[i].W;
    }
    int pr = prof_begin(PK_PC_FFT_FWD, prec, bfw, 0);
    STCHK(fft_grouped(prec, fw, false, "preconditioner FFT launch"));
    prof_end(pr);
    pr = prof_begin(PK_PC_GEMM, prec, bg, fl);
    STCHK(gemm_grouped(prec, gm, 1, "preconditioner product launch"));
    prof_end(pr);
    pr = prof_begin(PK_PC_FFT_INV, prec, bf, 0);
    STCHK(fft_grouped(prec, iv, true, "preconditioner IFFT launch"));
    prof_end(pr);
    return border_precond(items, prec);
}

// ------------------------------------------------------------------ setup

static void strang_weights(int N, std::vector<double>& w) {
    // lags -(N-1) .. N-1: weight 1 for 2|p| < N, 1/2 for 2|p| = N, 0 otherwise
    w.assign(2 * N - 1, 0.0);
    for (int p = -(N - 1); p < N; ++p) {
        const int a = p < 0 ? -p : p;
        w[p + N - 1] = 2 * a < N ? 1.0 : (2 * a == N ? 0.5 : 0.0);
    }
}

static mlfft_status build_array(Ctx* c, Array& a, const double2* Rdev) {
    const int Nx = a.Nx, Ny = a.Ny, b = a.b;
    const int bb = b * b;
    const int nly = 2 * Ny - 1, nlx = 2 * Nx - 1;
    hipStream_t s = c->stream;
    // spectra on the (2Ny) x (2Nx) grid
    Buf T(&c->alloc);
    const size_t tb = (size_t)nly * a.Px * bb * sizeof(double2);
    HIPCHK(T.ensure(tb), "spectra scratch");
    HIPCHK(a.G64.ensure((size_t)a.K * bb * sizeof(double2)), "spectra");
    HIPCHK(a.G32.ensure((size_t)a.K * bb * sizeof(float2)), "spectra");
    HIPCHK(a.G16.ensure((size_t)a.K * bb * sizeof(uint32_t)), "spectra");
    HIPCHK(launch_lag_dft_x(Rdev, (double2*)T.p, nly, nlx, -(Nx - 1), a.Px, nullptr, bb, s), "spectra x");
    HIPCHK(launch_lag_dft_y((double2*)T.p, (double2*)a.G64.p, nly, -(Ny - 1), a.Py, a.Px, nullptr, bb, s),
           "spectra y");
    HIPCHK(launch_cast_c64_to_c32((double2*)a.G64.p, (float2*)a.G32.p, (size_t)a.K * bb, s), "spectra cast");
    HIPCHK(launch_cast_c64_to_bf16((double2*)a.G64.p, (uint32_t*)a.G16.p, (size_t)a.K * bb, s), "spectra cast");
    // Strang block circulant on the Ny x Nx torus
    std::vector<double> wx, wy;
    strang_weights(Nx, wx);
    strang_weights(Ny, wy);
    Buf Wt(&c->alloc);
    HIPCHK(Wt.ensure((wx.size() + wy.size()) * sizeof(double)), "weights");
    HIPCHK(hipMemcpyAsync(Wt.p, wx.data(), wx.size() * sizeof(double), hipMemcpyHostToDevice, s), "weights");
    HIPCHK(hipMemcpyAsync((double*)Wt.p + wx.size(), wy.data(), wy.size() * sizeof(double),
                          hipMemcpyHostToDevice, s), "weights");
    const int Kp = Nx * Ny;
    Buf Sh(&c->alloc), Aw(&c->alloc), rc(&c->alloc), inf(&c->alloc);
    HIPCHK(Sh.ensure((size_t)Kp * bb * sizeof(double2)), "preconditioner scratch");
    HIPCHK(launch_lag_dft_x(Rdev, (double2*)T.p, nly, nlx, -(Nx - 1), Nx, (double*)Wt.p, bb, s), "strang x");
    HIPCHK(launch_lag_dft_y((double2*)T.p, (double2*)Sh.p, nly, -(Ny - 1), Ny, Nx, (double*)Wt.p + wx.size(), bb, s),
           "strang y");
    HIPCHK(a.S64.ensure((size_t)Kp * bb * sizeof(double2)), "preconditioner");
    HIPCHK(a.S32.ensure((size_t)Kp * bb * sizeof(float2)), "preconditioner");
    HIPCHK(a.S16.ensure((size_t)Kp * bb * sizeof(uint32_t)), "preconditioner");
    HIPCHK(rc.ensure((size_t)(Kp + 1) * sizeof(double)), "rcond");
    HIPCHK(inf.ensure((size_t)(Kp + 1) * sizeof(int)), "info");
    HIPCHK(launch_batched_inverse((double2*)Sh.p, (double2*)a.S64.p, (double*)rc.p, (int*)inf.p, Kp, b, s),
           "preconditioner inverse");
    // self block inverse
    HIPCHK(Aw.ensure((size_t)bb * sizeof(double2)), "self block");
    HIPCHK(a.K64.ensure((size_t)bb * sizeof(double2)), "self block");
    const double2* R00 = Rdev + ((size_t)(Ny - 1) * nlx + (Nx - 1)) * bb;
    HIPCHK(hipMemcpyAsync(Aw.p, R00, (size_t)bb * sizeof(double2), hipMemcpyDeviceToDevice, s), "self block");
    HIPCHK(launch_batched_inverse((double2*)Aw.p, (double2*)a.K64.p, (double*)rc.p + Kp, (int*)inf.p + Kp, 1, b, s),
           "self block inverse");
    std::vector<double> rcond(Kp + 1);
    std::vector<int> info(Kp + 1);
    HIPCHK(hipMemcpyAsync(rcond.data(), rc.p, (Kp + 1) * sizeof(double), hipMemcpyDeviceToHost, s), "rcond");
    HIPCHK(hipMemcpyAsync(info.data(), inf.p, (Kp + 1) * sizeof(int), hipMemcpyDeviceToHost, s), "info");
    HIPCHK(hipStreamSynchronize(s), "setup");
    if (info[Kp] != 0 || !(rcond[Kp] >= 1e-14))
        return c->fail(MLFFT_E_SINGULAR, "self block R_{0,0} is singular (rcond %.3e)", rcond[Kp]);
    std::vector<int> bad(Kp);
    a.pc_fallbacks = 0;
    a.pc_min_rcond = 1.0;
    for (int k = 0; k < Kp; ++k) {
        bad[k] = (info[k] != 0 || !(rcond[k] >= 1e-12)) ? 1 : 0;
        a.pc_fallbacks += bad[k];
        if (rcond[k] < a.pc_min_rcond) a.pc_min_rcond = rcond[k];
    }
    if (a.pc_fallbacks) {
        HIPCHK(hipMemcpyAsync(inf.p, bad.data(), Kp * sizeof(int), hipMemcpyHostToDevice, s), "fallback flags");
        HIPCHK(launch_fill_identity_fallback((double2*)a.S64.p, (double2*)a.K64.p, (int*)inf.p, Kp, b, s),
               "fallback");
    }
    HIPCHK(launch_cast_c64_to_c32((double2*)a.S64.p, (float2*)a.S32.p, (size_t)Kp * bb, s), "cast");
    HIPCHK(launch_cast_c64_to_bf16((double2*)a.S64.p, (uint32_t*)a.S16.p, (size_t)Kp * bb, s), "cast");
    HIPCHK(a.K32.ensure((size_t)bb * sizeof(float2)), "self block");
    HIPCHK(a.K16.ensure((size_t)bb * sizeof(uint32_t)), "self block");
    HIPCHK(launch_cast_c64_to_c32((double2*)a.K64.p, (float2*)a.K32.p, (size_t)bb, s), "cast");
    HIPCHK(launch_cast_c64_to_bf16((double2*)a.K64.p, (uint32_t*)a.K16.p, (size_t)bb, s), "cast");
    HIPCHK(hipStreamSynchronize(s), "setup");
    // scratch buffers (T, Sh, Aw, ...) are released by their destructors after the sync
    return MLFFT_OK;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

mlfft_status mlfft_create(int device, void* hip_stream, mlfft_alloc_fn alloc_fn, mlfft_free_fn free_fn, void* user,
                          mlfft_ctx* out) {
    if (!out) { g_create_error = "out is NULL"; return MLFFT_E_ARG; }
    *out = nullptr;
    if (!alloc_fn || !free_fn) { g_create_error = "alloc_fn and free_fn must not be NULL"; return MLFFT_E_ARG; }
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
        g_create_error = "invalid device or no HIP device";
        (void)hipGetLastError();
        return MLFFT_E_ARG;
    }
    e = hipSetDevice(device);
    if (e != hipSuccess) { g_create_error = hipGetErrorString(e); return MLFFT_E_HIP; }
    e = scratch_init(device);
    if (e != hipSuccess) { g_create_error = std::string("scratch set-up: ") + hipGetErrorString(e); return MLFFT_E_HIP; }
    Ctx* c = new Ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->alloc.fn = alloc_fn;
    c->alloc.fr = free_fn;
    c->alloc.user = user;
    for (Buf* b : {&c->spec_a, &c->spec_b, &c->task_dev, &c->solve_ws, &c->solve_ws2}) b->bind(&c->alloc);
    *out = c;
    return MLFFT_OK;
}

mlfft_status mlfft_destroy(mlfft_ctx ctx) {
    if (!ctx) return MLFFT_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->arrays) kv.second.release();
    ctx->release_workspaces();
    delete ctx;
    return MLFFT_OK;
}

const char* mlfft_last_error(mlfft_ctx ctx) {
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

mlfft_status mlfft_set_stream(mlfft_ctx ctx, void* hip_stream) {
    if (!ctx) return MLFFT_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return MLFFT_OK;
}

mlfft_status mlfft_set_blocks(mlfft_ctx ctx, int array_id, int Nx, int Ny, int b, const void* blocks,
                              int blocks_on_device) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (array_id < 0) return c->fail(MLFFT_E_ARG, "array_id must be >= 0");
    if (Nx < 1 || Ny < 1 || Nx > kMaxGrid || Ny > kMaxGrid)
        return c->fail(MLFFT_E_ARG, "Nx, Ny must be in [1, %d] (got %d, %d)", kMaxGrid, Nx, Ny);
    if (b < 1 || b > 256) return c->fail(MLFFT_E_ARG, "b must be in [1, 256] (got %d)", b);
    if (!blocks) return c->fail(MLFFT_E_ARG, "blocks is NULL");
    HIPCHK(hipSetDevice(c->device), "set device");
    const size_t nblk = (size_t)(2 * Ny - 1) * (2 * Nx - 1) * b * b;
    if (!blocks_on_device) {
        const double* h = (const double*)blocks;
        for (size_t i = 0; i < 2 * nblk; ++i)
            if (!std::isfinite(h[i])) return c->fail(MLFFT_E_ARG, "blocks contain a non-finite value at %zu", i / 2);
    }
    Buf R(&c->alloc);
    HIPCHK(R.ensure(nblk * sizeof(double2)), "block upload");
    HIPCHK(hipMemcpyAsync(R.p, blocks, nblk * sizeof(double2),
                          blocks_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
           "block upload");
    if (blocks_on_device) {
        Buf flag(&c->alloc);
        HIPCHK(flag.ensure(sizeof(int)), "flag");
        HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int), c->stream), "flag");
        HIPCHK(launch_nonfinite((const double*)R.p, 2 * nblk, (int*)flag.p, c->stream), "finite check");
        int hflag = 0;
        HIPCHK(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream), "flag");
        HIPCHK(hipStreamSynchronize(c->stream), "finite check");
        if (hflag) return c->fail(MLFFT_E_ARG, "blocks contain a non-finite value");
    }
    auto old = c->arrays.find(array_id);
    if (old != c->arrays.end()) {
        HIPCHK(hipStreamSynchronize(c->stream), "replace array");
        old->second.release();
        c->arrays.erase(old);
    }
    Array a;
    a.bind(&c->alloc);
    a.Nx = Nx; a.Ny = Ny; a.b = b;
    a.Px = 2 * Nx; a.Py = 2 * Ny; a.K = a.Px * a.Py;
    mlfft_status st = build_array(c, a, (const double2*)R.p);
    if (st != MLFFT_OK) { a.release(); return st; }
    a.R64 = std::move(R);           // kept for the direct solver and the row preconditioner
    c->arrays.emplace(array_id, std::move(a));
    return MLFFT_OK;
}

mlfft_status mlfft_drop_array(mlfft_ctx ctx, int array_id) {
    if (!ctx) return MLFFT_E_ARG;
    auto it = ctx->arrays.find(array_id);
    if (it == ctx->arrays.end()) return ctx->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    (void)hipStreamSynchronize(ctx->stream);
    it->second.release();
    ctx->arrays.erase(it);
    return MLFFT_OK;
}

mlfft_status mlfft_array_info(mlfft_ctx ctx, int array_id, mlfft_array_info_t* out) {
    if (!ctx || !out) return MLFFT_E_ARG;
    Array* a = ctx->find(array_id);
    if (!a) return ctx->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    out->Nx = a->Nx; out->Ny = a->Ny; out->b = a->b; out->Px = a->Px; out->Py = a->Py;
    out->pc_fallbacks = a->pc_fallbacks;
    out->pc_min_rcond = a->pc_min_rcond;
    out->device_bytes = a->bytes();
    out->Nc = a->Nc;
    return MLFFT_OK;
}

static const char* kProfNames[PK_COUNT] = {"mlfft_fwd_fft", "block_gemm", "mlfft_inv_fft", "precond_fwd_fft",
                                           "precond_gemm", "precond_inv_fft", "arnoldi", "net_forward",
                                           "net_backward", "border_gemm"};

mlfft_status mlfft_profile_enable(mlfft_ctx ctx, int enable) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    HIPCHK(hipStreamSynchronize(c->stream), "profile");
    c->prof_recs.clear();
    c->prof_used = 0;
    c->prof = enable != 0;
    return MLFFT_OK;
}

mlfft_status mlfft_profile_read(mlfft_ctx ctx, mlfft_kernel_stat* out, int max_out, int* n_out) {
    if (!ctx || !n_out || (max_out > 0 && !out)) return MLFFT_E_ARG;
    Ctx* c = ctx;
    HIPCHK(hipStreamSynchronize(c->stream), "profile");
    std::vector<mlfft_kernel_stat> agg;
    for (const ProfRec& r : c->prof_recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b), "profile event");
        mlfft_kernel_stat* hit = nullptr;
        for (auto& s : agg)
            if (strcmp(s.name, kProfNames[r.kind]) == 0 && s.prec == r.prec) hit = &s;
        if (!hit) {
            mlfft_kernel_stat s{};
            snprintf(s.name, sizeof s.name, "%s", kProfNames[r.kind]);
            s.prec = r.prec;
            agg.push_back(s);
            hit = &agg.back();
        }
        hit->launches += 1;
        hit->ms += ms;
        hit->bytes += r.bytes;
        hit->flops += r.flops;
    }
    *n_out = (int)agg.size();
    for (int i = 0; i < (int)agg.size() && i < max_out; ++i) out[i] = agg[i];
    return MLFFT_OK;
}

mlfft_status mlfft_matvec(mlfft_ctx ctx, int array_id, int W, const void* x, void* y, mlfft_prec prec) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (W < 0) return c->fail(MLFFT_E_ARG, "W must be >= 0");
    if (prec < MLFFT_FP64 || prec > MLFFT_FP32_BF16GEMM) return c->fail(MLFFT_E_ARG, "invalid precision");
    if (W == 0) return MLFFT_OK;
    if (!x || !y) return c->fail(MLFFT_E_ARG, "x or y is NULL");
    const size_t vb = a->Nt() * W * prec_elem_bytes(prec);
    if ((const char*)x < (const char*)y + vb && (const char*)y < (const char*)x + vb)
        return c->fail(MLFFT_E_ARG, "x and y overlap");
    HIPCHK(hipSetDevice(c->device), "set device");
    std::vector<MatvecItem> items(1);
    items[0] = MatvecItem{a, W, x, y, nullptr, 1.0, 0.0};
    return c->matvec_group(items, prec);
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    return (const char*)a < (const char*)b + nb && (const char*)b < (const char*)a + na;
}

mlfft_status mlfft_matvec_axpby(mlfft_ctx ctx, int array_id, int W, double alpha, const void* x, double beta,
                                const void* v, void* y, mlfft_prec prec) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (W < 0) return c->fail(MLFFT_E_ARG, "W must be >= 0");
    if (prec < MLFFT_FP64 || prec > MLFFT_FP32_BF16GEMM) return c->fail(MLFFT_E_ARG, "invalid precision");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return c->fail(MLFFT_E_ARG, "alpha and beta must be finite");
    if (W == 0) return MLFFT_OK;
    if (!x || !y) return c->fail(MLFFT_E_ARG, "x or y is NULL");
    const size_t vb = a->Nt() * W * prec_elem_bytes(prec);
    if (overlap(x, vb, y, vb)) return c->fail(MLFFT_E_ARG, "x and y overlap");
    if (v && overlap(v, vb, y, vb)) return c->fail(MLFFT_E_ARG, "v and y overlap");
    HIPCHK(hipSetDevice(c->device), "set device");
    std::vector<MatvecItem> items(1);
    items[0] = MatvecItem{a, W, x, y, v, alpha, v ? beta : 0.0};
    return c->matvec_group(items, prec);
}

mlfft_status mlfft_axpby(mlfft_ctx ctx, size_t n, double alpha, const void* x, double beta, const void* y,
                         int in_prec, void* out, int out_prec) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if ((in_prec != MLFFT_FP64 && in_prec != MLFFT_FP32) || (out_prec != MLFFT_FP64 && out_prec != MLFFT_FP32))
        return c->fail(MLFFT_E_ARG, "precisions must be MLFFT_FP64 or MLFFT_FP32");
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return c->fail(MLFFT_E_ARG, "alpha and beta must be finite");
    if (n == 0) return MLFFT_OK;
    if (!x || !out) return c->fail(MLFFT_E_ARG, "x or out is NULL");
    const size_t ib = n * prec_elem_bytes(in_prec), ob = n * prec_elem_bytes(out_prec);
    // out may be x or y itself (each element is read before it is written), but no partial overlap
    if (overlap(x, ib, out, ob) && !(x == out && ib == ob)) return c->fail(MLFFT_E_ARG, "x and out partially overlap");
    if (y && overlap(y, ib, out, ob) && !(y == out && ib == ob))
        return c->fail(MLFFT_E_ARG, "y and out partially overlap");
    HIPCHK(hipSetDevice(c->device), "set device");
    HIPCHK(launch_axpby(in_prec, x, y, alpha, beta, out_prec, out, n, c->stream), "axpby");
    return MLFFT_OK;
}

mlfft_status mlfft_precond_apply(mlfft_ctx ctx, int array_id, int kind, int W, const void* r, void* z,
                                 mlfft_prec prec) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (kind != 1 && kind != 2 && kind != 4) return c->fail(MLFFT_E_ARG, "preconditioner kind must be 1, 2 or 4");
    if (W < 0) return c->fail(MLFFT_E_ARG, "W must be >= 0");
    if (prec < MLFFT_FP64 || prec > MLFFT_FP32_BF16GEMM) return c->fail(MLFFT_E_ARG, "invalid precision");
    if (W == 0) return MLFFT_OK;
    if (!r || !z) return c->fail(MLFFT_E_ARG, "r or z is NULL");
    const size_t vb = a->Nt() * W * prec_elem_bytes(prec);
    if ((const char*)r < (const char*)z + vb && (const char*)z < (const char*)r + vb)
        return c->fail(MLFFT_E_ARG, "r and z overlap");
    HIPCHK(hipSetDevice(c->device), "set device");
    std::vector<MatvecItem> items(1);
    items[0] = MatvecItem{a, W, r, z, nullptr, 1.0, 0.0};
    return c->precond_group(items, kind, prec);
}

}  // extern "C"
