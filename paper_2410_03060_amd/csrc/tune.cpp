// Autotuning table shared by the product launchers of every discretisation.
#include "tune.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

namespace chaff {

namespace {
std::mutex g_mu;
std::vector<TuneEntry> g_tab;

bool same_key(const TuneEntry& a, const TuneEntry& b) {
    return a.nb == b.nb && a.n == b.n && a.nnzb == b.nnzb && a.s == b.s && a.prec == b.prec;
}

// Value of "key": in one JSON object text (numbers only), or nullptr.
const char* field(const std::string& obj, const char* key) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t p = obj.find(k);
    if (p == std::string::npos) return nullptr;
    const char* v = obj.c_str() + p + k.size();
    while (*v == ' ' || *v == '\t' || *v == '\n' || *v == '\r') ++v;
    return v;
}
}  // namespace

int tuned_variant(int nb, int64_t n, int64_t nnzb, int64_t s, int prec) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const TuneEntry& e : g_tab)
        if (e.nb == nb && e.n == n && e.nnzb == nnzb && e.s == s && e.prec == prec) return e.best;
    return -1;
}

void record_tuning(const TuneEntry& t) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (TuneEntry& e : g_tab)
        if (same_key(e, t)) {
            e = t;
            return;
        }
    g_tab.push_back(t);
}

std::string tune_json() {
    std::lock_guard<std::mutex> lk(g_mu);
    std::string out = "[";
    for (size_t i = 0; i < g_tab.size(); ++i) {
        const TuneEntry& e = g_tab[i];
        char line[640];
        int m = std::snprintf(line, sizeof line, "%s{\"nb\":%d,\"n\":%lld,\"nnzb\":%lld,\"s\":%lld,\"prec\":%d,\"best\":%d,\"ms\":[",
                              i ? "," : "", e.nb, (long long)e.n, (long long)e.nnzb, (long long)e.s, e.prec, e.best);
        for (int v = 0; v < TUNE_VARIANTS; ++v)
            m += std::snprintf(line + m, sizeof line - (size_t)m, "%s%.4f", v ? "," : "", e.ms[v]);
        std::snprintf(line + m, sizeof line - (size_t)m, "]}");
        out += line;
    }
    out += "]";
    return out;
}

int tune_merge_json(const std::string& text) {
    size_t a = text.find('[');
    if (a == std::string::npos) return -1;
    std::vector<TuneEntry> got;
    size_t p = a + 1;
    while (true) {
        const size_t o = text.find('{', p);
        if (o == std::string::npos) break;
        const size_t c = text.find('}', o);
        if (c == std::string::npos) return -1;
        const std::string obj = text.substr(o, c - o + 1);
        TuneEntry e{};
        const char* f;
        if (!(f = field(obj, "nb"))) return -1;
        e.nb = (int32_t)std::strtol(f, nullptr, 10);
        if (!(f = field(obj, "n"))) return -1;
        e.n = std::strtoll(f, nullptr, 10);
        if (!(f = field(obj, "nnzb"))) return -1;
        e.nnzb = std::strtoll(f, nullptr, 10);
        if (!(f = field(obj, "s"))) return -1;
        e.s = std::strtoll(f, nullptr, 10);
        if (!(f = field(obj, "prec"))) return -1;
        e.prec = (int32_t)std::strtol(f, nullptr, 10);
        if (!(f = field(obj, "best"))) return -1;
        e.best = (int32_t)std::strtol(f, nullptr, 10);
        if (e.best < 0 || e.best >= TUNE_VARIANTS || e.n < 1 || e.s < 1 || e.nnzb < 0 || (e.prec != 0 && e.prec != 1))
            return -1;
        if ((f = field(obj, "ms")) && *f == '[') {
            const char* q = f + 1;
            for (int v = 0; v < TUNE_VARIANTS; ++v) {
                char* end = nullptr;
                e.ms[v] = std::strtod(q, &end);
                if (end == q) break;
                q = end;
                while (*q == ',' || *q == ' ' || *q == '\n') ++q;
            }
        }
        got.push_back(e);
        p = c + 1;
    }
    for (const TuneEntry& e : got) record_tuning(e);
    return (int)got.size();
}

}  // namespace chaff
