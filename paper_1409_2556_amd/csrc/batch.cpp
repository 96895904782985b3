// Batches of problems: one host thread per problem drives that problem's
// handle and stream, so the shifted systems of grids of different shapes
// run concurrently on the GPU.  Nothing couples the problems (each
// right-hand side has its own basis, Section 3), so no device
// synchronisation between them is needed.
#include <hip/hip_runtime.h>

#include <set>
#include <string>
#include <thread>
#include <vector>

#include "lt_internal.h"

namespace {

constexpr int kMaxItems = 64;

template <typename Item>
int check_items(const Item* items, int n, bool (*uses_net)(const Item&)) {
    if (!items || n < 1 || n > kMaxItems) {
        lt::set_last_error("batch: need 1..64 items");
        return LT_EINVAL;
    }
    std::set<const lt_handle*> seen;
    std::set<const void*> nets;
    for (int i = 0; i < n; ++i) {
        const lt_handle* h = items[i].h;
        if (!h) {
            lt::set_last_error("batch: item " + std::to_string(i) + " has no handle");
            return LT_EINVAL;
        }
        if (!seen.insert(h).second) {
            lt::set_last_error("batch: handle of item " + std::to_string(i) + " appears twice");
            return LT_EINVAL;
        }
        if (uses_net(items[i]) && h->unet && !nets.insert(h->unet).second) {
            lt::set_last_error("batch: the network of item " + std::to_string(i) + " serves another item");
            return LT_EINVAL;
        }
    }
    return LT_OK;
}

// Run fn(i) for every item on its own thread (item 0 on the caller's) and
// combine the statuses; the caller's last error becomes the first failing
// item's message.
template <typename Fn>
int run_items(int n, const std::vector<int>& devices, int* status, Fn fn) {
    std::vector<std::string> msg(n);
    auto work = [&](int i) {
        if (hipSetDevice(devices[i]) != hipSuccess) {
            status[i] = LT_EHIP;
            msg[i] = "hipSetDevice failed";
            return;
        }
        status[i] = fn(i);
        if (status[i] < 0) msg[i] = lt_last_error();
    };
    std::vector<std::thread> threads;
    threads.reserve(n - 1);
    int caller_dev = 0;
    (void)hipGetDevice(&caller_dev);
    try {
        for (int i = 1; i < n; ++i) threads.emplace_back(work, i);
    } catch (...) {
        for (auto& t : threads) t.join();
        lt::set_last_error("batch: could not start threads");
        return LT_ENOMEM;
    }
    work(0);
    for (auto& t : threads) t.join();
    (void)hipSetDevice(caller_dev);
    int worst = LT_OK;
    for (int i = 0; i < n; ++i) {
        if (status[i] < 0) {
            lt::set_last_error("batch item " + std::to_string(i) + ": " + msg[i]);
            return status[i];
        }
        if (status[i] > 0) worst = status[i];
    }
    if (worst == LT_OK) lt::set_last_error("");
    return worst;
}

bool solve_uses_net(const lt_solve_item& it) { return it.opts && it.opts->precond == LT_PRECOND_UNET_GMG; }
bool adjoint_uses_net(const lt_adjoint_item& it) { return it.opts && it.opts->precond == LT_PRECOND_UNET_GMG; }

}  // namespace

extern "C" {

int lt_solve_batch(lt_solve_item* items, int n) {
    LT_TRY(check_items<lt_solve_item>(items, n, solve_uses_net));
    std::vector<int> dev(n), status(n, LT_OK);
    for (int i = 0; i < n; ++i) dev[i] = items[i].h->device;
    int rc = run_items(n, dev, status.data(), [items](int i) {
        lt_solve_item& it = items[i];
        return lt_solve(it.h, it.src, it.times, it.ntimes, it.contour, it.receivers, it.opts, it.phi_out,
                        it.stats);
    });
    for (int i = 0; i < n; ++i) items[i].status = status[i];
    return rc;
}

int lt_adjoint_batch(lt_adjoint_item* items, int n) {
    LT_TRY(check_items<lt_adjoint_item>(items, n, adjoint_uses_net));
    std::vector<int> dev(n), status(n, LT_OK);
    for (int i = 0; i < n; ++i) dev[i] = items[i].h->device;
    int rc = run_items(n, dev, status.data(), [items](int i) {
        lt_adjoint_item& it = items[i];
        return lt_adjoint(it.h, it.src, it.receivers, it.times, it.ntimes, it.contour, it.opts, it.dlnK, it.dlnS,
                          it.stats);
    });
    for (int i = 0; i < n; ++i) items[i].status = status[i];
    return rc;
}

}  // extern "C"
