// Per-frequency block product: planning, tuning table and dispatch (kernels in
// bgemm_impl.h, instantiated per precision in bgemm_f32.hip, bgemm_f64.hip and
// bgemm_bf16.hip so that the build compiles them in parallel).
#include "bgemm_impl.h"
#include "bgemm_launch.h"

namespace mlfft {

int gemm_bp(int prec, int b) {
    // padded reduction size: a multiple of 8 (FP32/FP64) or 16 (BF16)
    const int q = prec == PBF16 ? 16 : 8;
    int bp = (b + q - 1) / q * q;
    if (bp < q) bp = q;
    return bp;
}

static GemmShape g_shape_override[3][33];      // [prec][bp/8]; waves == 0: not tuned
static GemmShape g_shape_pc16[33];             // bf16 preconditioner product [bp/8]; waves == 0: default
// workgroups a launch of the frequency kernel aims at; 0: 512 for form 3, the device's
// CU count for form 5
static int g_pc_wg_target = 0;

void gemm_set_pc_wg_target(int n) { if (n >= 1 && n <= (1 << 20)) g_pc_wg_target = n; }

// compute units of the current device (cached per device)
static int device_cus() {
    static int cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

static GemmShape default_shape(int prec, int bp) {
    // FP64 from b = 33 (three 16-row slices): the flat three-product kernel with
    // direct-to-LDS half-reduction tiles
    if (prec == P64) return bp >= 40 ? GemmShape{4, 16, 4} : GemmShape{8, bp > 128 ? 16 : 32, 0};
    // FP32 from b = 97 (seven 16-row slices): the flat three-product kernel with
    // direct-to-LDS tiles (odd b falls back to the register-staged flat kernel)
    if (prec == P32) return bp >= 104 ? GemmShape{8, 16, 4} : GemmShape{8, bp > 160 ? 32 : 64, 0};
    // BF16: the eight-wave flat kernel (32-column tiles) for b >= 97, the four-wave one
    // (16-column tiles) for b >= 33, see launch_shape
    return GemmShape{8, 32, 2};
}

GemmShape gemm_shape(int prec, int bp, int tag) {
    if (tag) {
        if (prec == P64) return GemmShape{4, 16, 2};
        // the FP32 preconditioner product takes the tile shape tuned for the MLFFT
        // product of the same b when that is an eight-wave flat shape
        const GemmShape& o = g_shape_override[prec][bp / 8];
        if (prec == P32 && (o.m3 == 2 || o.m3 == 4) && o.waves == 8) return o;
        // the bf16 preconditioner product: each X tile staged once for all row slices of
        // its frequency, the (frequency, tile) items split evenly over about one workgroup
        // per CU (form 5), for padded b in 112..208, unless a shape was imported for it
        // (below 112 the flat kernels are faster, beyond 208 the stationary fragments spill)
        if (prec == PBF16)
            return g_shape_pc16[bp / 8].waves ? g_shape_pc16[bp / 8]
                                              : (bp >= 112 && bp <= 208) ? GemmShape{8, 32, 5} : GemmShape{8, 32, 2};
        return GemmShape{8, 32, 2};
    }
    const GemmShape& o = g_shape_override[prec][bp / 8];
    return o.waves ? o : default_shape(prec, bp);
}

void gemm_set_shape(int prec, int bp, int waves, int nt, int m3) {
    if (prec < 0 || prec > 2 || bp < 8 || bp > 256 || bp % 8) return;
    if (waves == 0) { g_shape_override[prec][bp / 8] = GemmShape{0, 0, 0}; return; }    // back to the default
    // BF16 has the eight-row kernel (m3 = 0) and the flat kernel with eight waves and
    // 32-column tiles or four waves and 16-column tiles
    if (prec == PBF16 && (m3 == 1 || (m3 == 2 && !((waves == 8 && nt == 32) || (waves == 4 && nt == 16))) ||
                          ((m3 == 3 || m3 == 5) && !(waves == 8 && nt == 32 && bp <= 208)) || m3 == 4 || m3 > 5))
        return;
    // form 4: the flat kernel with direct-to-LDS tiles, 16-column tiles, eight waves (FP32)
    // or four (FP64)
    if (prec != PBF16 && m3 > 2 && !(m3 == 4 && nt == 16 && waves == (prec == P32 ? 8 : 4))) return;
    g_shape_override[prec][bp / 8] = GemmShape{waves, nt, m3};
}

void gemm_set_pc_shape(int bp, int waves, int nt, int m3) {
    if (bp < 16 || bp > 256 || bp % 16) return;
    g_shape_pc16[bp / 8] = waves ? GemmShape{waves, nt, m3} : GemmShape{0, 0, 0};
}

bool bf16_spectrum_ok(const int* b, int n) {
    // the preconditioner product of these b (one padded b) reads bf16 spectra when it
    // runs form 5 with pairs: every b even
    if (n <= 0) return false;
    const int bp = gemm_bp(PBF16, b[0]);
    if (gemm_shape(PBF16, bp, 1).m3 != 5) return false;
    for (int i = 0; i < n; ++i)
        if ((b[i] & 1) || gemm_bp(PBF16, b[i]) != bp) return false;
    return true;
}

void gemm_get_shape(int prec, int bp, int* waves, int* nt, int* m3) {
    const GemmShape s = gemm_shape(prec, bp, 0);
    *waves = s.waves;
    *nt = s.nt;
    *m3 = s.m3;
}

static int bp_max_of(int prec, const GemmTask* tasks, int ntasks) {
    int bpm = 0;
    for (int i = 0; i < ntasks; ++i) bpm = std::max(bpm, gemm_bp(prec, tasks[i].b));
    return bpm;
}

// workgroups of one task: one per (frequency, row group), frequencies padded to a
// multiple of the XCD count; the flat three-product kernel (m3 == 2) deals the
// K * ceil(b/16) (frequency, slice) items to eight waves per workgroup
static int task_blocks(const GemmTask& t, const GemmShape& sh) {
    if (sh.m3 == 3) return t.K * t.mgroups;
    if (sh.m3 == 5) return t.mgroups;
    if (sh.m3 == 2 || sh.m3 == 4) return (t.K * ((t.b + 15) / 16) + sh.waves - 1) / sh.waves;
    return ((t.K + kXcd - 1) / kXcd) * kXcd * t.mgroups;
}

// The flat kernel stages at most two frequencies per workgroup, which holds when
// eight consecutive slices never cover three frequencies: ceil(b / 16) >= 7 for
// every task of the launch.  Otherwise the three-product kernel with one
// workgroup per row group is used.
static GemmShape launch_shape(int prec, const GemmTask* tasks, int ntasks, int tag, int bpm) {
    GemmShape sh = gemm_shape(prec, bpm, tag);
    if (sh.m3 == 4) {
        // the waves' consecutive slices span at most two frequencies (see below); FP32
        // direct-to-LDS tiles move two complex values per lane: every b even.  Otherwise
        // the flat kernel with register-staged tiles.
        bool ok = true;
        for (int i = 0; i < ntasks; ++i)
            ok = ok && (tasks[i].b + 15) / 16 >= sh.waves - 1 && (prec != P32 || (tasks[i].b & 1) == 0);
        if (!ok) sh = prec == P32 ? GemmShape{8, 16, 2} : GemmShape{4, 16, 2};
    }
    if (sh.m3 == 2 || sh.m3 == 4) {
        int bmin = 1 << 30;
        for (int i = 0; i < ntasks; ++i) bmin = std::min(bmin, tasks[i].b);
        // waves - 1 consecutive slices must not reach a third frequency
        if ((bmin + 15) / 16 < sh.waves - 1) {
            // bf16: the four-wave flat kernel down to 3 slices (b >= 33), a third faster than
            // the eight-row kernel at b = 64 and 96; below that the eight-row kernel
            if (prec == PBF16 && sh.waves == 8 && (bmin + 15) / 16 >= 3) sh = GemmShape{4, 16, 2};
            else sh = prec == P32 ? GemmShape{8, 32, 1} : prec == P64 ? GemmShape{8, bpm > 128 ? 16 : 32, 0}
                                                        : GemmShape{8, 64, 0};
        }
    }
    return sh;
}

void plan_gemm_tasks(int prec, GemmTask* tasks, int ntasks, int tag, int* grid, int* bp_max) {
    int g = 0;
    const int bpm = bp_max_of(prec, tasks, ntasks);
    const GemmShape sh = launch_shape(prec, tasks, ntasks, tag, bpm);
    const int rows = sh.m3 ? 16 : 8;
    // form 5: the (frequency, column tile) items of all tasks split over about one
    // workgroup per CU, each task taking a share proportional to its items
    long long items = 0;
    const int target5 = g_pc_wg_target ? g_pc_wg_target : device_cus();
    if (sh.m3 == 5)
        for (int i = 0; i < ntasks; ++i) items += (long long)tasks[i].K * ((tasks[i].W + sh.nt - 1) / sh.nt);
    for (int i = 0; i < ntasks; ++i) {
        GemmTask& t = tasks[i];
        const int nslices = (t.b + rows - 1) / rows;
        t.mgroups = (nslices + sh.waves - 1) / sh.waves;
        if (sh.m3 == 3) {
            // one frequency per workgroup; its columns split so that the launch has at
            // least the target number of workgroups, each split reading G once more
            const int tiles = (t.W + sh.nt - 1) / sh.nt;
            const int target = g_pc_wg_target ? g_pc_wg_target : 512;
            t.mgroups = std::max(1, std::min(tiles, (target + t.K - 1) / std::max(t.K, 1)));
        }
        if (sh.m3 == 5) {
            const long long mine = (long long)t.K * ((t.W + sh.nt - 1) / sh.nt);
            const long long share = items > 0 ? (target5 * mine + items - 1) / items : 1;
            t.mgroups = (int)std::max(1LL, std::min(mine, share));
        }
        t.block_begin = g;
        g += task_blocks(t, sh);
    }
    *grid = g;
    *bp_max = bpm;
}

hipError_t launch_bgemm(int prec, const GemmTask* th, const GemmTask* td, int ntasks, int tag, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    int grid = 0;
    const int bpm = bp_max_of(prec, th, ntasks);
    const GemmShape sh = launch_shape(prec, th, ntasks, tag, bpm);
    for (int i = 0; i < ntasks; ++i) {
        const int end = th[i].block_begin + task_blocks(th[i], sh);
        if (end > grid) grid = end;
    }
    if (grid == 0) return hipSuccess;
    const GemmTask* dt = ntasks > 1 ? td : nullptr;
    const int n = ntasks > 1 ? ntasks : 0;
    if (prec == P64) return launch_bgemm_f64(bpm, sh, tag, th[0], dt, n, grid, s);
    if (prec == P32) return launch_bgemm_f32(bpm, sh, tag, th[0], dt, n, grid, s);
    GemmShape s16 = sh;
    int nx16 = 0;
    for (int i = 0; i < ntasks; ++i) nx16 += th[i].x16 ? 1 : 0;
    if (s16.m3 == 5) {
        bool ok = true;
        for (int i = 0; i < ntasks; ++i)
            ok = ok && (th[i].b & 1) == 0 && (reinterpret_cast<uintptr_t>(th[i].X) & 15) == 0;
        s16.pairs = ok ? 1 : 0;
    }
    // bf16 spectra are only read by the pair-moving form-5 kernel, and by all tasks of a
    // launch or none (the caller decides per padded b with bf16_spectrum_ok)
    if (nx16 && (nx16 != ntasks || !s16.pairs)) return hipErrorInvalidValue;
    s16.x16 = nx16 ? 1 : 0;
    return launch_bgemm_bf16(bpm, s16, tag, th[0], dt, n, grid, s);
}

}  // namespace mlfft
