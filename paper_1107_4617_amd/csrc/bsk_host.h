// Host-side helpers shared by the C ABI translation units of libbsk.
#pragma once

#include <memory>

#include "../../include/bsk.h"
#include "bsk_internal.h"

namespace bsk {
namespace host {

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// Workspace slots, one per kind of use, so a buffer whose contents are cached
// across calls (the polynomial kernel's coefficient table, the patch filter's
// weights) is never written by another kind of call.
enum WsSlot {
    kWsAcc = 0,        // multi-pass accumulators: forward, patch, polynomial (rewritten by every call)
    kWsTrainAcc = 1,   // training-forward multi-pass accumulators
    kWsBwdTrain = 2,   // out and saved planes when the adjoint recomputes the training forward
    kWsBwdRed = 3,     // per-workgroup partial sums of the sigma_r gradient
    kWsBwdAcc = 4,     // adjoint multi-pass accumulators
    kWsPhase = 5,      // spatial-kernel phase tables (rewritten by every call)
    kWsPolyTab = 6,    // polynomial-kernel coefficient tables (cached)
    kWsPatchTab = 7,   // two-pixel-patch weight table (cached)
    kWsBatchTab = 8,   // batched descriptor and weight tables (uploaded by every call)
    kWsBatchAcc = 9    // batched multi-pass accumulators
};
// Grow-only device buffer per (device, stream, slot).  *gen (nullable)
// receives the buffer's allocation generation, unique across the process, so
// a cache keyed on it notices a reallocation even at the same address.
// Requests beyond the workspace limit (bsk_set_workspace_limit) fail with
// BSK_ENOMEM.
int get_ws(void *stream, int slot, size_t bytes, void **out, unsigned long long *gen = nullptr);
int device_cus();
bool finite_pos(double x);

// A validated single-image request: order, plan, clamped radii, launch shape.
struct Resolved {
    int N;
    int prec;
    int kahan;
    int pitch_in, pitch_out;
    int rh, rv;
    int block;
    int kc;        // orders per pass of the kernel the request runs
    int S;
    bsk::Plan plan;        // raised-cosine range kernel (unused for the polynomial one)
    bsk::SpatialPlan sp;   // Ns = 0: the box
    int range_kernel;      // bsk_range_kernel
    std::shared_ptr<const bsk::PolyPlan> poly;   // polynomial range kernel
    int poly_pairs;        // channel pairs of the polynomial kernel, ceil((K + 1) / 2)
};

// The kernel family a request is resolved for: its pass sizes and residency
// set the orders per pass and the segment height.
enum Kind { kForward = 0, kTrain = 1, kBackward = 2, kPatch2 = 3 };
// nimg: the images of one size launched together (they share the round of
// resident workgroups the segment height is chosen for).
int resolve(int H, int W, int radius, float sigma_r, float T, const bsk_options *opt, Resolved *r,
            int kind = kForward, int nimg = 1);
// Orders per pass from a kernel family's full pass, a smaller one (0: half
// the full one) and optionally a third size between them (0: none): the one
// with the lower estimated cost for K orders.
int pick_chunk(int K, int full, int small = 0, int mid = 0);
// The cheapest of n pass sizes by the same cost.
int pick_chunk_of(int K, const int *sizes, int n);
// Plan of the polynomial range kernel, cached per (N, sigma_r, T, eps).
std::shared_ptr<const bsk::PolyPlan> poly_plan(int N, double sigma_r, double T, double eps);
// Fills the launch arguments; the weights are padded with zeros to a multiple
// of `kc` (the pass size of the kernel that will run).
void fill_args(bsk::StripArgs *a, const Resolved &r, int H, int W, int kc);
int nblocks(const Resolved &r, int H, int W);
bool overlap(const void *a, size_t na, const void *b, size_t nb);

// Tuned launch shape for a single-image forward request, if the autotuner has
// measured one for this (radius, orders, H, W, precision); returns false if not.
bool tuned_shape(int rh, int K, int H, int W, int prec, int *block, int *S, int *kc);

}  // namespace host
}  // namespace bsk
