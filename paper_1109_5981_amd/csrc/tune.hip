// tune.hip -- the process-wide table of tuned launch shapes, keyed by
// (phase, dtype, rows bucket, cols), with its text form for export and
// import.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace lsrn {

namespace {

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int64_t>, int> g_tune;

const char *phase_name(int p) { return p == TUNE_SWEEP ? "sweep" : "?"; }
const char *dtype_name(int d) { return d == 1 ? "f32" : "f64"; }

}  // namespace

int rows_bucket(int64_t rows) {
    int b = 0;
    while (b < 62 && ((int64_t)1 << b) < rows) ++b;
    return b;
}

bool tune_lookup(const TuneKey &k, int &value) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(k.phase, k.dtype, k.rows_log2, k.cols));
    if (it == g_tune.end()) return false;
    value = it->second;
    return true;
}

void tune_store(const TuneKey &k, int value) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(k.phase, k.dtype, k.rows_log2, k.cols)] = value;
}

}  // namespace lsrn

extern "C" {

size_t lsrn_tune_export(char *buf, size_t len) {
    std::ostringstream os;
    {
        std::lock_guard<std::mutex> lk(lsrn::g_tune_mu);
        for (const auto &e : lsrn::g_tune)
            os << lsrn::phase_name(std::get<0>(e.first)) << ' ' << lsrn::dtype_name(std::get<1>(e.first))
               << ' ' << std::get<2>(e.first) << ' ' << std::get<3>(e.first) << ' ' << e.second << '\n';
    }
    const std::string t = os.str();
    if (buf && len > t.size()) std::memcpy(buf, t.c_str(), t.size() + 1);
    return t.size() + 1;
}

lsrn_status lsrn_tune_import(const char *text) {
    if (!text) return LSRN_E_INVALID;
    std::istringstream is(text);
    std::string line;
    std::vector<std::pair<lsrn::TuneKey, int>> add;
    while (std::getline(is, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::istringstream ls(line);
        std::string ph, dt, extra;
        int rb = -1, value = 0;
        long long cols = -1;
        if (!(ls >> ph >> dt >> rb >> cols >> value) || (ls >> extra)) return LSRN_E_INVALID;
        if (ph != "sweep" || (dt != "f64" && dt != "f32") || rb < 0 || rb > 62 || cols <= 0 ||
            value < 1 || value > 64)
            return LSRN_E_INVALID;
        lsrn::TuneKey k;
        k.phase = lsrn::TUNE_SWEEP;
        k.dtype = dt == "f32" ? 1 : 0;
        k.rows_log2 = rb;
        k.cols = cols;
        add.emplace_back(k, value);
    }
    for (const auto &e : add) lsrn::tune_store(e.first, e.second);
    return LSRN_OK;
}

void lsrn_tune_clear(void) {
    std::lock_guard<std::mutex> lk(lsrn::g_tune_mu);
    lsrn::g_tune.clear();
}

}  // extern "C"
