// Tile table lookup for the TTVc sweep.
#include <mutex>
#include <vector>

#include "tuning.h"

namespace hoscf {

namespace {

struct Entry {
    int dtype;
    int order;
    int64_t dims[kMaxOrder];
    int64_t tiling[6];
};

std::mutex g_mu;
std::vector<Entry> g_table;

bool same_shape(const Entry& e, const hoscf_tensor& T) {
    if (e.dtype != T.dtype || e.order != T.order) return false;
    for (int i = 0; i < T.order; ++i)
        if (e.dims[i] != T.dims[i]) return false;
    return true;
}

}  // namespace

SweepTuning tuning_from(const int64_t* t) {
    SweepTuning s;
    s.target_wg = std::max<int64_t>(0, t[0]);
    s.bp_min = std::max<int64_t>(1, t[1]);
    s.lr = (int)t[2];
    s.align = (int)t[3];
    s.mb = (int)t[4];
    s.nw = (int)t[5];
    return s;
}

SweepTuning lookup_tuning(const hoscf_tensor& T) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const Entry& e : g_table)
            if (same_shape(e, T)) return tuning_from(e.tiling);
    }
    // Built-in rule, from level-1 sweeps measured on MI355X (FP32 800^3,
    // 200^4, 64^5; BF16 and FP8 64^5): with the row-by-row refill, full rows
    // per lane group and 8 waves (128 rows of a workgroup for FP32) were
    // fastest at every order: the partial outputs per m-tile, written while
    // T streams, cost far more per byte than the reads, and bigger tiles
    // write fewer of them.
    (void)T;
    SweepTuning s;
    s.mb = 0;
    s.nw = 8;
    return s;
}

}  // namespace hoscf

using namespace hoscf;

extern "C" int hoscf_tune_set(const hoscf_tensor* T, const int64_t* tiling) {
    if (!T || T->order < 2 || T->order > kMaxOrder || T->dtype < 0 || T->dtype > 3) return HOSCF_INVALID_ARG;
    if (tiling) {
        if (tiling[0] < 0 || tiling[1] < 0 || tiling[2] < 0 || tiling[2] > 64 || (tiling[2] & (tiling[2] - 1)) ||
            (tiling[3] != 0 && tiling[3] != 1) || tiling[4] < 0 || (tiling[5] != 0 && tiling[5] != 4 && tiling[5] != 8))
            return HOSCF_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_table.size(); ++i)
        if (same_shape(g_table[i], *T)) {
            g_table.erase(g_table.begin() + (long)i);
            break;
        }
    if (tiling) {
        Entry e{};
        e.dtype = T->dtype;
        e.order = T->order;
        for (int i = 0; i < T->order; ++i) e.dims[i] = T->dims[i];
        for (int i = 0; i < 6; ++i) e.tiling[i] = tiling[i];
        g_table.push_back(e);
    }
    return HOSCF_OK;
}

extern "C" void hoscf_tune_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}
