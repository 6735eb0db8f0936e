// Process-wide tuning table for the sweep schedule (queries per lane, key-splitting
// waves, blocks per CU, merge mode), keyed by (d, size class of the query set,
// size class of the key set).
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "ct_internal.h"

namespace ct {

namespace {
struct Entry {
    int R, WS, bpc, sep, us;
};
std::mutex g_mu;
std::map<std::tuple<int, int, int>, Entry> g_table;

int size_class(int64_t n) {
    int c = 0;
    while ((int64_t(1) << c) < n) ++c;
    return c;  // ceil(log2 n)
}
}  // namespace

Schedule schedule_for(int d, int64_t nq, int64_t nk) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find({d, size_class(nq), size_class(nk)});
        if (it != g_table.end())
            return Schedule{it->second.R, it->second.WS, it->second.bpc, it->second.sep};
    }
    // untuned default: more queries per lane and fewer key-splitting waves when
    // there are many queries
    Schedule s{2, 4, 16, 1};
    if (nq < 65536) s = Schedule{2, 2, 4, 1};
    if (nq < 8192) s = Schedule{4, 4, 2, 1};
    (void)d;
    (void)nk;
    return s;
}

bool tuning_lookup(int d, int qclass, int kclass, Schedule& out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find({d, qclass, kclass});
    if (it == g_table.end()) return false;
    out = Schedule{it->second.R, it->second.WS, it->second.bpc, it->second.sep};
    return true;
}

void tuning_record(int d, int64_t nq, int64_t nk, const Schedule& sc, int us) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[{d, size_class(nq), size_class(nk)}] =
        Entry{sc.R, sc.WS, sc.blocks_per_cu, sc.sep, us};
}

}  // namespace ct

using namespace ct;

extern "C" int32_t ct_tuning_count(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int32_t)g_table.size();
}

extern "C" ct_status ct_tuning_entry(int32_t i, int32_t* out8) {
    if (!out8) return fail(CT_E_ARG, "out8 is null");
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int32_t)g_table.size()) return fail(CT_E_ARG, "entry %d out of range", i);
    auto it = g_table.begin();
    std::advance(it, i);
    out8[0] = std::get<0>(it->first);
    out8[1] = std::get<1>(it->first);
    out8[2] = std::get<2>(it->first);
    out8[3] = it->second.R;
    out8[4] = it->second.WS;
    out8[5] = it->second.bpc;
    out8[6] = it->second.sep;
    out8[7] = it->second.us;
    return CT_OK;
}

extern "C" ct_status ct_tuning_save(const char* path) {
    if (!path) return fail(CT_E_ARG, "path is null");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(CT_E_ARG, "cannot open %s for writing", path);
    std::lock_guard<std::mutex> lk(g_mu);
    std::fprintf(f, "# d qclass kclass R WS blocks_per_cu separate_merge us\n");
    for (auto& kv : g_table)
        std::fprintf(f, "%d %d %d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
                     std::get<2>(kv.first), kv.second.R, kv.second.WS, kv.second.bpc,
                     kv.second.sep, kv.second.us);
    std::fclose(f);
    return CT_OK;
}

extern "C" ct_status ct_tuning_load(const char* path) {
    if (!path) return fail(CT_E_ARG, "path is null");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(CT_E_ARG, "cannot open %s", path);
    char line[256];
    std::lock_guard<std::mutex> lk(g_mu);
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int d, qc, kc, R, ws, b, sep, us;
        const int nf = std::sscanf(line, "%d %d %d %d %d %d %d %d", &d, &qc, &kc, &R, &ws, &b,
                                   &sep, &us);
        if (nf <= 0) continue;  // blank line
        if (nf != 8 || (d != 2 && d != 3) || (R != 1 && R != 2 && R != 4 && R != 8) ||
            (ws != 1 && ws != 2 && ws != 4) || b < 1 || b > 16 || (sep != 0 && sep != 1)) {
            std::fclose(f);
            return fail(CT_E_ARG, "bad tuning entry: %s", line);
        }
        g_table[{d, qc, kc}] = Entry{R, ws, b, sep, us};
    }
    std::fclose(f);
    return CT_OK;
}

extern "C" void ct_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}
