// Learned preconditioner: network state and the C ABI of its forward, backward and training.
#include "lib.h"

struct Net {};

bool Ctx::net_ready() const { return net != nullptr; }

void Ctx::net_release() {
    delete net;
    net = nullptr;
}

mlfft_status Ctx::net_correct(const mlfft::Array*, int, const void*, void*, int, int*) {
    return fail(MLFFT_E_STATE, "no network");
}
