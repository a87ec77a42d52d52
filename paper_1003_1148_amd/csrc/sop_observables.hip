// Force-spectroscopy observables of the pulling and indentation protocols
// (Section IV.B): running averages of a force trace, the peak (unfolding)
// force, and the virial estimate of the temperature.  Host code: these act
// on recorded traces, not on the per-step path.
#include <cmath>
#include <cstdint>
#include <vector>

#include "sop.h"

namespace {

// Double-double accumulator (Knuth's TwoSum): the running prefix sums of a
// long trace keep about 106 bits, so a window sum taken as the difference of
// two prefixes is accurate to the last bit of a double whatever the trace
// length.
struct DD {
    double hi = 0.0, lo = 0.0;
};

inline DD dd_add(DD a, double b)
{
    const double s = a.hi + b;
    const double bp = s - a.hi;
    const double e = (a.hi - (s - bp)) + (b - bp);
    const double lo = a.lo + e;
    const double hi = s + lo;
    return DD{hi, lo - (hi - s)};
}

inline double dd_diff(DD a, DD b)
{
    // (a.hi - b.hi) by TwoSum, then the low parts
    const double s = a.hi - b.hi;
    const double bp = s - a.hi;
    const double e = (a.hi - (s - bp)) + (-b.hi - bp);
    return s + (e + (a.lo - b.lo));
}

}  // namespace

extern "C" {

sop_status sop_running_average(const double *y, int64_t n, int32_t w, double *out)
{
    if (!y || !out || w < 1 || n < (int64_t)w)
        return SOP_E_ARG;
    DD head, tail;  // prefix sums up to k + w and up to k
    for (int32_t j = 0; j < w; ++j)
        head = dd_add(head, y[j]);
    const double inv = 1.0 / (double)w;
    for (int64_t k = 0;; ++k) {
        out[k] = dd_diff(head, tail) * inv;
        if (k + w >= n)
            break;
        head = dd_add(head, y[k + w]);
        tail = dd_add(tail, y[k]);
    }
    return SOP_OK;
}

sop_status sop_peak_force(const double *f, int64_t n, int32_t w, double *peak, int64_t *index)
{
    if (!f || !peak || !index || w < 1 || n < (int64_t)w)
        return SOP_E_ARG;
    std::vector<double> a((size_t)(n - w + 1));
    sop_running_average(f, n, w, a.data());
    int64_t best = 0;
    for (int64_t k = 1; k < (int64_t)a.size(); ++k)
        if (a[k] > a[best])
            best = k;
    *peak = a[best];
    *index = best;
    return SOP_OK;
}

sop_status sop_virial_temperature(const double *virial, int64_t n_records, int64_t n_res, double kB,
                                  double *T)
{
    if (!virial || !T || n_records < 1 || n_res < 2 || !(kB > 0.0))
        return SOP_E_ARG;
    DD sum;
    for (int64_t k = 0; k < n_records; ++k)
        sum = dd_add(sum, virial[k]);
    const double mean = (sum.hi + sum.lo) / (double)n_records;
    *T = -mean / (3.0 * (double)(n_res - 1) * kB);
    return SOP_OK;
}

}  // extern "C"
