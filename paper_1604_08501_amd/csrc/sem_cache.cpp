// Plan cache file of the mixed-order batch autotuner (see sem_cache.hpp).
#include "sem_cache.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace semcache {

namespace {

constexpr size_t kMaxKey = 256;

// Value of "name": <number> inside one entry's body, or NAN if absent or not
// a number.
double number(const std::string& body, const char* name)
{
    const std::string key = std::string("\"") + name + "\"";
    const size_t k = body.find(key);
    if (k == std::string::npos)
        return NAN;
    const size_t c = body.find(':', k + key.size());
    if (c == std::string::npos)
        return NAN;
    const char* p = body.c_str() + c + 1;
    char* end = nullptr;
    const double v = strtod(p, &end);
    return end == p ? NAN : v;
}

bool in_range(double v, double lo, double hi)
{
    return std::isfinite(v) && v >= lo && v <= hi;
}

}  // namespace

std::map<std::string, Entry> read(const std::string& path)
{
    std::map<std::string, Entry> m;
    FILE* f = fopen(path.c_str(), "rb");
    if (!f)
        return m;
    std::string s;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0)
        s.append(buf, n);
    fclose(f);
    size_t pos = 0;
    while (true) {
        const size_t k0 = s.find('"', pos);
        if (k0 == std::string::npos)
            break;
        const size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos)
            break;
        const size_t ob = s.find('{', k1);
        const size_t cb = s.find('}', k1);
        if (ob == std::string::npos || cb == std::string::npos || cb < ob)
            break;
        const std::string body = s.substr(ob, cb - ob);
        const double epb = number(body, "epb"), lay = number(body, "layout"),
                     us = number(body, "us");
        if (k1 - k0 - 1 <= kMaxKey && in_range(epb, 1, 4096) && in_range(lay, 0, 15) &&
            in_range(us, 0, 1e12)) {
            Entry e;
            e.epb = (int)epb;
            e.lay = (int)lay;
            e.us = us;
            m[s.substr(k0 + 1, k1 - k0 - 1)] = e;
        }
        pos = cb + 1;
    }
    return m;
}

void write(const std::string& path, const std::map<std::string, Entry>& m)
{
    const std::string tmp = path + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f)
        return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m)
        fprintf(f, "  \"%s\": {\"epb\": %d, \"layout\": %d, \"us\": %.3f}%s\n", kv.first.c_str(),
                kv.second.epb, kv.second.lay, kv.second.us, ++i < m.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path.c_str());
}

}  // namespace semcache
