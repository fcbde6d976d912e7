// Launchers of the learned-correction kernels (net.hip).
#pragma once
#include "internal.h"

namespace mlfft {

hipError_t n_normalise(const float2* y, size_t N, int W, int npix, int b, int cpad, float2* yhat, unsigned short* a0,
                       double* scale, double2* phase, hipStream_t s);
hipError_t n_target(const float2* e, size_t N, int W, int npix, int b, int cpad, const double* scale,
                    const double2* phase, float* tgt, hipStream_t s);
hipError_t n_conv_fwd(const unsigned short* act, const unsigned short* wt, void* out, int nimg, int H, int Wd,
                      int cin, int cout, int bf16_relu, hipStream_t s);
hipError_t n_finish(const float2* y, const float2* yhat, const float* netout, size_t N, int W, int b, int cpad,
                    const double* scale, const double2* phase, float2* z, int* fallback, hipStream_t s);
hipError_t n_loss_grad(const float2* yhat, const float* out, const float* tgt, size_t N, int W, int b, int cpad,
                       float* gout, double* loss, hipStream_t s);
hipError_t n_dgrad(const float* g, const unsigned short* wt, const unsigned short* amask, float* gin, int nimg, int H,
                   int Wd, int cin, int cout, hipStream_t s);
// the weight gradient sums per-chunk partials (part: n_wgrad_chunks(P, cin, cout) x cout x 9 x cin floats)
int n_wgrad_chunks(long P, int cin, int cout);
hipError_t n_wgrad(const float* g, const unsigned short* act, float* dw, float* part, int nimg, int H, int Wd, int cin,
                   int cout, hipStream_t s);
hipError_t n_adam(float* wmaster, float* m, float* v, const float* dw, unsigned short* wbf, int cin, int cout, int cinp,
                  float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t n_pack_weights(const float* wmaster, unsigned short* wbf, int cin, int cout, int cinp, int coutp,
                          hipStream_t s);
hipError_t n_unpack_grad(const float* dwp, float* dw, int cin, int cout, int cinp, hipStream_t s);
hipError_t n_pack_nhwc(const float* x, unsigned short* a, long npix_total, int c, int cpad, hipStream_t s);
hipError_t n_unpack_nhwc(const float* o, float* x, long npix_total, int c, int cpad, hipStream_t s);

}  // namespace mlfft
