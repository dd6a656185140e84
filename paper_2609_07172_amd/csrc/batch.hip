// Solves of several independent problems (uneven grids) in one call: each
// problem runs cylpoisson_solve on a stream and a host thread of its own, so
// the small problems' launches fill the GPU beside the large ones'.
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "cp_internal.h"

namespace cp {

namespace {

// One stream and one host thread per problem; each solve runs exactly as alone.
int solve_streams(cylpoisson_plan* const* plans, const double* const* rho, double* const* phi, int count,
                  double tol, hipStream_t s, int* statuses) {
    std::vector<hipStream_t> st(count, nullptr);
    std::vector<hipEvent_t> ev(count, nullptr);
    std::vector<int> res(count, CYLPOISSON_OK);
    std::vector<std::string> msg(count);
    hipEvent_t start = nullptr;
    int status = CYLPOISSON_OK;
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(start, s) != hipSuccess) {
        (void)hipGetLastError();
        set_error("batch: cannot order the problems after the caller's stream");
        if (start) (void)hipEventDestroy(start);
        return CYLPOISSON_EHIP;
    }
    for (int i = 0; i < count && status == CYLPOISSON_OK; ++i) {
        int prev = 0;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(plans[i]->device);
        if (hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess ||
            hipStreamWaitEvent(st[i], start, 0) != hipSuccess) {
            (void)hipGetLastError();
            set_error("batch: cannot create the stream of problem %d", i);
            status = CYLPOISSON_EHIP;
        }
        (void)hipSetDevice(prev);
    }
    if (status == CYLPOISSON_OK) {
        std::vector<std::thread> threads;
        threads.reserve(count);
        for (int i = 0; i < count; ++i)
            threads.emplace_back([&, i] {
                res[i] = cylpoisson_solve(plans[i], rho[i], phi[i], tol, st[i]);
                msg[i] = cylpoisson_last_error();
                if (hipEventRecord(ev[i], st[i]) != hipSuccess) res[i] = CYLPOISSON_EHIP;
            });
        for (auto& t : threads) t.join();
        for (int i = 0; i < count; ++i) {
            if (statuses) statuses[i] = res[i];
            if (hipStreamWaitEvent(s, ev[i], 0) != hipSuccess) res[i] = CYLPOISSON_EHIP;
        }
        // the batch status: the first error, else NOT_CONVERGED if any, else OK
        for (int i = 0; i < count; ++i)
            if (res[i] < 0) {
                set_error("batch problem %d: %s", i, msg[i].c_str());
                status = res[i];
                break;
            }
        if (status == CYLPOISSON_OK)
            for (int i = 0; i < count; ++i)
                if (res[i] == CYLPOISSON_NOT_CONVERGED) {
                    set_error("batch problem %d: %s", i, msg[i].c_str());
                    status = CYLPOISSON_NOT_CONVERGED;
                    break;
                }
    }
    for (int i = 0; i < count; ++i) {
        if (st[i]) (void)hipStreamSynchronize(st[i]);
        if (st[i]) (void)hipStreamDestroy(st[i]);
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
    (void)hipEventDestroy(start);
    return status;
}

}  // namespace

}  // namespace cp

using namespace cp;

extern "C" {

int cylpoisson_solve_batch(cylpoisson_plan* const* plans, const double* const* rho, double* const* phi,
                           int count, double tol, void* stream, int* statuses) {
    if (count < 0 || (count > 0 && (!plans || !rho || !phi))) {
        set_error("batch arrays must not be NULL and count must be >= 0");
        return CYLPOISSON_EINVAL;
    }
    for (int i = 0; i < count; ++i)
        for (int j = 0; j < i; ++j)
            if (plans[i] == plans[j] || !plans[i]) {
                set_error("batch entry %d: plans must be distinct and not NULL", i);
                return CYLPOISSON_EINVAL;
            }
    if (count > 0 && !plans[0]) {
        set_error("batch entry 0: plans must be distinct and not NULL");
        return CYLPOISSON_EINVAL;
    }
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        set_error("tol must be a positive finite number");
        return CYLPOISSON_EINVAL;
    }
    return solve_streams(plans, rho, phi, count, tol, static_cast<hipStream_t>(stream), statuses);
}

}  // extern "C"
