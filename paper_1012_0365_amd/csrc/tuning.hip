// Split-K plans of the generic GEMM kernels (the W-products): how many
// workgroups a product of a given shape should be spread over. Fewer splits
// write fewer partial sums; more keep every CU busy on small products. The
// best count depends on the shape and was measured on the device by
// paper_1012_0365_amd/autotune.py, which wrote tuned_plans.inc: for each
// precision, product size sqrt(M K) and block width N, the fastest of the
// candidate targets. A shape takes the entry nearest to it (log scale); the
// table is fixed at build time, so every run makes the same choice.
#include <atomic>
#include <cmath>

#include "blws_common.h"

namespace blws {
namespace {

struct TunedPlan {
    int prec, size, n, target;
};

const TunedPlan kTuned[] = {
#include "tuned_plans.inc"
};

std::atomic<int> g_override{0};

}  // namespace

void set_plan_override(int target) { g_override.store(target < 0 ? 0 : target); }

int plan_target(int prec, int M, int N, int K, int fallback)
{
    const int o = g_override.load();
    if (o > 0) return o;
    // the table covers the W-products: a long side on both M and K
    if (M < 256 || K < 256 || N < 1 || N > 1024) return fallback;
    const double ls = 0.5 * std::log((double)M * (double)K), ln = std::log((double)N);
    double best = 1e300;
    int t = fallback;
    for (const TunedPlan& e : kTuned) {
        if (e.prec != prec) continue;
        const double ds = ls - std::log((double)e.size), dn = ln - std::log((double)e.n);
        const double d = ds * ds + dn * dn;
        if (d < best) {
            best = d;
            t = e.target;
        }
    }
    return t;
}

}  // namespace blws

extern "C" int blws_set_plan_target(int target)
{
    if (target < 0 || target > 65536) return BLWS_EINVAL;
    blws::set_plan_override(target);
    return BLWS_OK;
}
