// Autotuner: times the candidate launch shapes of the hot kernels on the
// actual shape of an array (its K, b, Nx, Ny and a given W) with HIP events and
// keeps the fastest for the rest of the process.  Choices can be exported as
// text and imported again (a cache keyed by kernel, precision and shape).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lib.h"

using namespace mlfft;

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return c->hip_fail(e_, what);  \
    } while (0)

namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() { (void)hipEventCreate(&a); (void)hipEventCreate(&b); }
    ~Timer() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
};

std::string g_report;

// A later candidate replaces the current best only if it is faster by more than
// this margin, so that timing noise does not flip the choice between runs.
const double kTuneMargin = 0.98;

}  // namespace

// time `reps` runs of fn (after one warm-up run); returns mean ms or a negative value on error
template<typename F>
static double time_it(Ctx* c, int reps, F fn) {
    Timer t;
    if (fn() != hipSuccess) return -1.0;
    (void)hipEventRecord(t.a, c->stream);
    for (int i = 0; i < reps; ++i)
        if (fn() != hipSuccess) return -1.0;
    (void)hipEventRecord(t.b, c->stream);
    if (hipEventSynchronize(t.b) != hipSuccess) return -1.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    return ms / reps;
}

extern "C" {

mlfft_status mlfft_autotune(mlfft_ctx ctx, int array_id, int W, int prec, int reps) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    if (W < 1 || reps < 1 || prec < 0 || prec > 2) return c->fail(MLFFT_E_ARG, "bad autotune arguments");
    HIPCHK(hipSetDevice(c->device), "set device");
    const int eb = prec_elem_bytes(prec);
    const size_t sb = (size_t)a->K * a->b * W * eb;
    HIPCHK(c->spec_a.ensure(sb), "tuning workspace");
    HIPCHK(c->spec_b.ensure(sb), "tuning workspace");
    HIPCHK(hipMemsetAsync(c->spec_a.p, 0, sb, c->stream), "tuning workspace");
    HIPCHK(hipMemsetAsync(c->spec_b.p, 0, sb, c->stream), "tuning workspace");
    char line[256];
    std::string rep;
    // ---- block product of the MLFFT matvec
    const int bp = gemm_bp(prec, a->b);
    const int ntc[3] = {prec == P64 ? 16 : 32, prec == P64 ? 32 : 64, 16};
    int bw = 0, bn = 0, bm = 0;
    double best = 1e30;
    if (prec != PBF16) {
        for (int m3 : {0, 1, 2, 4}) for (int waves : {4, 8}) {
            if (m3 == 1 && prec != P32) continue;
            // form 4: the flat kernel with direct-to-LDS tiles, 16 columns, eight waves (FP32,
            // even b) or four (FP64)
            if (m3 == 4 && (prec == PBF16 || waves != (prec == P32 ? 8 : 4) || (prec == P32 && (a->b & 1)) ||
                            (a->b + 15) / 16 < waves - 1))
                continue;
            // the flat three-product kernels run eight or four waves (FP32, four with
            // 16-column tiles only) or four (FP64)
            if (m3 == 2 && prec == P64 && waves != 4) continue;
            for (int ci = 0; ci < 3; ++ci) {
                const int nt = ntc[ci];
                // nt 16 is only a shape of the flat FP32 kernel (eight waves: double-buffered
                // tiles; four waves: single-buffered, two workgroups per CU)
                if (ci == 2 && !((m3 == 2 || m3 == 4) && prec == P32)) continue;
                if (m3 == 4 && (nt != 16 || (prec == P64 && ci == 2))) continue;
                // four waves: only where the eight-wave flat kernel cannot run (fewer than
                // seven 16-row slices); at larger b its tiles are re-read from HBM more
                if (m3 == 2 && prec == P32 && waves == 4 && (nt != 16 || (a->b + 15) / 16 >= 7)) continue;
                if (m3 == 2 && prec == P64 && nt != 16) continue;
                if (m3 == 2 && prec == P32 && nt == 64) continue;
                gemm_set_shape(prec, bp, waves, nt, m3);
                GemmTask g{};
                g.G = prec == P64 ? a->G64.p : a->G32.p;
                g.X = c->spec_a.p; g.Y = c->spec_b.p; g.K = a->K; g.b = a->b; g.W = W;
                g.gstride = (long)a->b * a->b;
                int grid, bpm;
                plan_gemm_tasks(prec, &g, 1, 0, &grid, &bpm);
                const double ms = time_it(c, reps, [&]() { return launch_bgemm(prec, &g, nullptr, 1, 0, c->stream); });
                snprintf(line, sizeof line, "block_gemm prec=%d b=%d K=%d W=%d waves=%d nt=%d m3=%d: %.4f ms\n", prec,
                         a->b, a->K, W, waves, nt, m3, ms);
                rep += line;
                if (ms > 0 && ms < kTuneMargin * best) { best = ms; bw = waves; bn = nt; bm = m3; }
            }
        }
        if (bw) gemm_set_shape(prec, bp, bw, bn, bm);
    }
    // ---- forward / inverse 2-D FFT (MLFFT grid and preconditioner torus), each
    // direction on its own: tile kind (one-pass or half-height, padded grids) x m-chunk
    const int fprec = prec == P64 ? P64 : P32;
    for (int pad : {1, 0}) {
        for (int dir : {0, 1}) {
            int bestcm = 0, besthalf = -1;
            double bestms = 1e30;
            for (int half : {0, 1}) {
                if (half && !pad) continue;
                fft_set_choice(fprec, pad, dir, a->Nx, a->Ny, a->b, 0, half);
                if (fft_use_half(fprec, pad, dir, a->Nx, a->Ny, a->b) != (half != 0)) continue;
                const int cmax = fft_max_cm(fprec, pad, half, a->Nx, a->Ny, a->b);
                for (int cm = 1; cm <= cmax; cm *= 2) {
                    fft_set_choice(fprec, pad, dir, a->Nx, a->Ny, a->b, cm, half);
                    FftTask f{};
                    f.in = dir ? c->spec_a.p : c->spec_b.p;
                    f.out = dir ? c->spec_b.p : c->spec_a.p;
                    f.alpha = 1.0;
                    f.Nx = a->Nx; f.Ny = a->Ny; f.b = a->b; f.W = W; f.pad = pad;
                    int grid, block;
                    size_t lds;
                    plan_fft_tasks(fprec, &f, 1, dir, &grid, &block, &lds);
                    if (f.cm != cm) continue;
                    const double ms = time_it(c, reps, [&]() {
                        return dir ? launch_fft_inv(fprec, &f, nullptr, 1, c->stream)
                                   : launch_fft_fwd(fprec, &f, nullptr, 1, c->stream);
                    });
                    snprintf(line, sizeof line, "fft %s prec=%d pad=%d Nx=%d Ny=%d b=%d W=%d half=%d cm=%d: %.4f ms\n",
                             dir ? "inv" : "fwd", fprec, pad, a->Nx, a->Ny, a->b, W, half, cm, ms);
                    rep += line;
                    if (ms > 0 && ms < kTuneMargin * bestms) { bestms = ms; bestcm = cm; besthalf = half; }
                }
            }
            fft_set_choice(fprec, pad, dir, a->Nx, a->Ny, a->b, bestcm, besthalf);
        }
    }
    g_report = rep;
    return MLFFT_OK;
}

// Text of the choices currently in force for an array shape, one "key value" per line,
// and the timings of the last mlfft_autotune() call.
mlfft_status mlfft_tune_report(mlfft_ctx ctx, int array_id, char* buf, size_t n) {
    if (!ctx || !buf || n == 0) return MLFFT_E_ARG;
    Ctx* c = ctx;
    Array* a = c->find(array_id);
    if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_id);
    std::string s;
    char line[256];
    for (int prec : {0, 1}) {
        int w, nt, m3;
        gemm_get_shape(prec, gemm_bp(prec, a->b), &w, &nt, &m3);
        snprintf(line, sizeof line, "gemm %d %d %d %d %d\n", prec, gemm_bp(prec, a->b), w, nt, m3);
        s += line;
        for (int pad : {1, 0})
            for (int dir : {0, 1}) {
                int cm, half;
                fft_get_choice(prec, pad, dir, a->Nx, a->Ny, a->b, &cm, &half);
                snprintf(line, sizeof line, "fftshape %d %d %d %d %d %d %d %d\n", prec, pad, dir, a->Nx, a->Ny, a->b,
                         cm, half);
                s += line;
            }
    }
    s += g_report;
    snprintf(buf, n, "%s", s.c_str());
    return MLFFT_OK;
}

// Apply choices in the format of mlfft_tune_report ("gemm", "gemmpc", "gemmpcwg",
// "fftshape" and the older "fftcm" lines; other lines are ignored).
mlfft_status mlfft_tune_import(mlfft_ctx ctx, const char* text) {
    if (!ctx || !text) return MLFFT_E_ARG;
    Ctx* c = ctx;
    const char* p = text;
    while (*p) {
        const char* e = strchr(p, '\n');
        std::string ln(p, e ? (size_t)(e - p) : strlen(p));
        int a1, a2, a3, a4, a5, a6, a7, a8;
        if (sscanf(ln.c_str(), "gemm %d %d %d %d %d", &a1, &a2, &a3, &a4, &a5) == 5) {
            const bool reset = a3 == 0 && a4 == 0 && a5 == 0;       // back to the default shape
            const bool ok = a1 >= 0 && a1 <= 2 && a2 >= 8 && a2 <= 256 && a2 % 8 == 0 && (reset || ((a3 == 4 || a3 == 8) &&
                            (a4 == 16 || a4 == 32 || a4 == 64) &&
                            (a5 == 0 || (a5 == 1 && a1 == 1) || (a5 == 2 && a1 == 1 && a3 == 8 && a4 == 32) ||
                             (a5 == 2 && a1 == 1 && a3 == 8 && a4 == 16) || (a5 == 2 && a1 == 1 && a3 == 4 && a4 == 16) ||
                             (a5 == 2 && a1 == 0 && a3 == 4 && a4 == 16) || (a5 == 2 && a1 == 2 && a3 == 8 && a4 == 32) ||
                             (a5 == 2 && a1 == 2 && a3 == 4 && a4 == 16) || (a5 == 4 && a1 == 1 && a3 == 8 && a4 == 16) ||
                             (a5 == 4 && a1 == 0 && a3 == 4 && a4 == 16))));
            if (!ok) return c->fail(MLFFT_E_ARG, "bad tuning line: %s", ln.c_str());
            gemm_set_shape(a1, a2, a3, a4, a5);
        } else if (sscanf(ln.c_str(), "gemmpc %d %d %d %d %d", &a1, &a2, &a3, &a4, &a5) == 5) {
            // the bf16 preconditioner product: form 3 (one frequency per workgroup, padded b up
            // to 208) or form 2 (the flat kernel, eight waves, 32-column tiles); waves 0 restores
            // the default
            const bool ok = a1 == 2 && a2 >= 16 && a2 <= 256 && a2 % 16 == 0 &&
                            ((a3 == 8 && a4 == 32 && (a5 == 2 || ((a5 == 3 || a5 == 5) && a2 <= 208))) || a3 == 0);
            if (!ok) return c->fail(MLFFT_E_ARG, "bad tuning line: %s", ln.c_str());
            gemm_set_pc_shape(a2, a3, a4, a5);
        } else if (sscanf(ln.c_str(), "gemmpcwg %d", &a1) == 1) {
            if (a1 < 1 || a1 > (1 << 20)) return c->fail(MLFFT_E_ARG, "bad tuning line: %s", ln.c_str());
            gemm_set_pc_wg_target(a1);
        } else if (sscanf(ln.c_str(), "fftshape %d %d %d %d %d %d %d %d", &a1, &a2, &a3, &a4, &a5, &a6, &a7, &a8) == 8) {
            if (a1 < 0 || a1 > 1 || a2 < 0 || a2 > 1 || a3 < 0 || a3 > 1 || a4 < 1 || a5 < 1 || a6 < 1 ||
                a7 < 0 || a7 > 64 || a8 < -1 || a8 > 1 || (a8 == 1 && !a2))
                return c->fail(MLFFT_E_ARG, "bad tuning line: %s", ln.c_str());
            fft_set_choice(a1, a2, a3, a4, a5, a6, a7, a8);
        } else if (sscanf(ln.c_str(), "fftcm %d %d %d %d %d %d", &a1, &a2, &a3, &a4, &a5, &a6) == 6) {
            // both directions, default tile kind
            if (a1 < 0 || a1 > 1 || a2 < 0 || a2 > 1 || a6 < 0 || a6 > 64)
                return c->fail(MLFFT_E_ARG, "bad tuning line: %s", ln.c_str());
            for (int dir : {0, 1}) fft_set_choice(a1, a2, dir, a3, a4, a5, a6, -1);
        }
        if (!e) break;
        p = e + 1;
    }
    return MLFFT_OK;
}

}  // extern "C"
