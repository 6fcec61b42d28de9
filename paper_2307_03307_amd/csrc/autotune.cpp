// Autotuner of batched layouts.  A layout (tile sizes and launch shape of the
// batched passes) is picked by coordinate descent: each field in turn takes
// every value of its candidate list with the other fields at their best so
// far, and the program rates each candidate by a timed run of the batch
// itself.  Results are remembered per (program, device, precision, batch
// shape) for the life of the process and, when a cache file is named,
// appended to it as text (and looked up there first), one layout per line:
//   <key> <tile_edges> <tile_vertices> <workgroups_per_cu> <search_launches> <rate>
// The last line of a key wins; lines that do not parse are skipped.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "host.h"

namespace mwu {

namespace {

std::mutex g_mutex;
std::map<std::string, std::pair<mwu_batch_layout, double>> g_known;

int half_octave(int64_t v)   // floor(2 log2 v), 0 for v < 1
{
    return v < 1 ? 0 : (int)std::floor(2.0 * std::log2((double)v));
}

int32_t *field(mwu_batch_layout &L, int f)
{
    switch (f) {
    case 0: return &L.tile_edges;
    case 1: return &L.tile_vertices;
    case 2: return &L.workgroups_per_cu;
    default: return &L.search_launches;
    }
}

}  // namespace

bool layout_valid(const mwu_batch_layout &L)
{
    auto tile_ok = [](int32_t t) { return t >= BLOCK && t <= 65536 && t % BLOCK == 0; };
    return tile_ok(L.tile_edges) && tile_ok(L.tile_vertices) && L.workgroups_per_cu >= 1 &&
           L.workgroups_per_cu <= 16 && L.search_launches >= 1 && L.search_launches <= 4;
}

mwu_batch_layout default_layout()
{
    mwu_batch_layout L;
    std::memset(&L, 0, sizeof(L));
    L.tile_edges = BLOCK * 8;
    L.tile_vertices = BLOCK * 16;
    L.workgroups_per_cu = 8;
    L.search_launches = 2;
    L.source = MWU_LAYOUT_DEFAULT;
    return L;
}

std::string tune_key(const char *program, bool fp32, int device, int num_cus, int32_t count, int64_t nv,
                     int64_t ne, int64_t max_ne)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        for (char &ch : arch)
            if (ch == ' ' || ch == '\t') ch = '_';
    }
    std::ostringstream k;
    k << "mwu1/" << program << '/' << (fp32 ? "mixed" : "fp64") << '/' << arch << "/cu" << num_cus << "/b"
      << half_octave(count) << "/v" << half_octave(nv) << "/e" << half_octave(ne) << "/emax"
      << half_octave(max_ne);
    return k.str();
}

bool tune_lookup(const std::string &key, const char *path, mwu_batch_layout *L, double *rate)
{
    if (path && *path) {   // a named file is read first: it may hold a newer record
        std::ifstream in(path);
        std::string line;
        bool found = false;
        while (in && std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            mwu_batch_layout c = default_layout();
            double r = 0.0;
            if (!(ls >> k >> c.tile_edges >> c.tile_vertices >> c.workgroups_per_cu >> c.search_launches >> r))
                continue;
            if (k != key || !layout_valid(c)) continue;
            *L = c;
            *rate = r;
            found = true;
        }
        if (found) {
            std::lock_guard<std::mutex> g(g_mutex);
            g_known[key] = {*L, *rate};
            return true;
        }
    }
    {
        std::lock_guard<std::mutex> g(g_mutex);
        auto it = g_known.find(key);
        if (it == g_known.end()) return false;
        *L = it->second.first;
        *rate = it->second.second;
    }
    if (path && *path) tune_store(key, path, *L, *rate);   // the file lacked it: append the record
    return true;
}

void tune_store(const std::string &key, const char *path, const mwu_batch_layout &L, double rate)
{
    {
        std::lock_guard<std::mutex> g(g_mutex);
        g_known[key] = {L, rate};
    }
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    if (!out) return;   // an unwritable cache only loses the record
    char buf[96];
    std::snprintf(buf, sizeof(buf), " %d %d %d %d %.6e\n", L.tile_edges, L.tile_vertices, L.workgroups_per_cu,
                  L.search_launches, rate);
    out << key << buf;
}

mwu_batch_layout tune_descent(const mwu_batch_layout &start, const std::vector<std::vector<int32_t>> &cands,
                              const std::function<double(const mwu_batch_layout &)> &rate, int *timed,
                              double *best_rate)
{
    std::map<std::vector<int32_t>, double> seen;
    auto key = [](mwu_batch_layout &L) {
        return std::vector<int32_t>{L.tile_edges, L.tile_vertices, L.workgroups_per_cu, L.search_launches};
    };
    mwu_batch_layout best = start;
    double best_r = -1.0;
    *timed = 0;
    for (int f = 0; f < 4 && f < (int)cands.size(); ++f) {
        for (int32_t v : cands[f]) {
            mwu_batch_layout c = best;
            *field(c, f) = v;
            if (!layout_valid(c)) continue;
            const std::vector<int32_t> id = key(c);
            double r;
            auto it = seen.find(id);
            if (it != seen.end()) {
                r = it->second;
            } else {
                r = rate(c);
                seen[id] = r;
                ++*timed;
            }
            if (r > best_r) {
                best_r = r;
                best = c;
            }
        }
    }
    *best_rate = std::max(0.0, best_r);
    return best;
}

}  // namespace mwu
