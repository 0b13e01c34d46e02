// Plan selection: the leaf size L and the dense/FFT crossover s* of a handle.
//
// The recursive solve's two free parameters trade latency against bandwidth:
// L sets how many sequential leaf launches there are (N / L) and how much
// in-leaf history each leaf step carries; s* decides which level products
// run as dense Toeplitz-block products (launch- and latency-bound) and which
// as circulant-embedded FFT products (section 3.1; bandwidth-bound).  The
// best values depend on the width M (which fixes the leaf's configuration)
// and on the arithmetic of the products.  They are measured by the tuner
// (paper_1710_11593_amd/tune.py, which times whole solves through the C ABI)
// and looked up here:
//   1. options leaf / crossover > 0 (or crossover < 0: FFT at every level)
//      are used as given;
//   2. otherwise the plan cache, a JSON file written by the tuner, is read
//      unless FRACSOLVE_TUNE=0: $FRACSOLVE_TUNE_CACHE, else
//      $XDG_CACHE_HOME/fracsolve/plan.json, else ~/.cache/fracsolve/plan.json;
//   3. otherwise (no file, unreadable, malformed, or no matching entry) the
//      built-in table below, which holds the tuner's measurements on MI355X.
//
// Cache format:
//   {"fracsolve_plan": 1,
//    "entries": [{"precision": 0, "equation": 0, "m_max": 128,
//                 "leaf": 8, "crossover": 64}, ...]}
// An entry applies to handles of that precision and equation whose widest
// instance has M <= m_max; the entry with the smallest such m_max wins.  A
// file with any malformed entry is ignored as a whole.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fracsolve.h"
#include "plan.hpp"

namespace fs {

namespace {

// ---------------------------------------------------------------- a small JSON reader
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0.0;
    std::string str;
    std::vector<JVal> items;                          // ARR
    std::vector<std::pair<std::string, JVal>> fields;  // OBJ
    const JVal *get(const char *key) const
    {
        for (auto &f : fields)
            if (f.first == key) return &f.second;
        return nullptr;
    }
};

struct JParser {
    const char *p, *end;
    int depth = 0;
    bool ok = true;
    void ws()
    {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool lit(const char *s)
    {
        size_t n = strlen(s);
        if ((size_t)(end - p) >= n && memcmp(p, s, n) == 0) {
            p += n;
            return true;
        }
        return false;
    }
    bool string(std::string &out)
    {
        if (p >= end || *p != '"') return false;
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (p >= end) return false;
                const char c = *p;
                if (c == 'u') return false;  // not needed by the cache format
                out.push_back(c == 'n' ? '\n' : c == 't' ? '\t' : c);
            } else {
                if ((unsigned char)*p < 0x20) return false;
                out.push_back(*p);
            }
            ++p;
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool value(JVal &v)
    {
        if (++depth > 16) return false;
        ws();
        if (p >= end) return false;
        bool r = true;
        if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
            } else {
                for (;;) {
                    ws();
                    std::string key;
                    JVal item;
                    if (!string(key)) return false;
                    ws();
                    if (p >= end || *p != ':') return false;
                    ++p;
                    if (!value(item)) return false;
                    v.fields.emplace_back(std::move(key), std::move(item));
                    ws();
                    if (p < end && *p == ',') {
                        ++p;
                        continue;
                    }
                    if (p < end && *p == '}') {
                        ++p;
                        break;
                    }
                    return false;
                }
            }
        } else if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
            } else {
                for (;;) {
                    JVal item;
                    if (!value(item)) return false;
                    v.items.push_back(std::move(item));
                    ws();
                    if (p < end && *p == ',') {
                        ++p;
                        continue;
                    }
                    if (p < end && *p == ']') {
                        ++p;
                        break;
                    }
                    return false;
                }
            }
        } else if (*p == '"') {
            v.kind = JVal::STR;
            r = string(v.str);
        } else if (lit("true")) {
            v.kind = JVal::BOOL;
            v.num = 1;
        } else if (lit("false")) {
            v.kind = JVal::BOOL;
        } else if (lit("null")) {
            v.kind = JVal::NUL;
        } else {
            char *q = nullptr;
            std::string tok;
            while (p < end && (isdigit((unsigned char)*p) || strchr("+-.eE", *p))) tok.push_back(*p++);
            if (tok.empty()) return false;
            v.kind = JVal::NUM;
            v.num = strtod(tok.c_str(), &q);
            r = q && *q == '\0';
        }
        --depth;
        return r;
    }
};

bool read_file(const std::string &path, std::string &out)
{
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return false;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) {
        out.append(buf, n);
        if (out.size() > (1u << 20)) {  // a plan file is a few KB
            fclose(f);
            return false;
        }
    }
    fclose(f);
    return true;
}

bool as_int(const JVal *v, int lo, int hi, int *out)
{
    if (!v || v->kind != JVal::NUM) return false;
    const double d = v->num;
    if (!(d >= lo && d <= hi) || d != (double)(int)d) return false;
    *out = (int)d;
    return true;
}

// Entries of a cache file; false if the file is missing or malformed.
bool load_cache(const std::string &path, std::vector<PlanEntry> &out)
{
    std::string text;
    if (!read_file(path, text)) return false;
    JParser jp{text.data(), text.data() + text.size()};
    JVal root;
    if (!jp.value(root)) return false;
    jp.ws();
    if (jp.p != jp.end || root.kind != JVal::OBJ) return false;
    int version = 0;
    if (!as_int(root.get("fracsolve_plan"), 1, 1, &version)) return false;
    const JVal *ents = root.get("entries");
    if (!ents || ents->kind != JVal::ARR) return false;
    std::vector<PlanEntry> got;
    for (const JVal &e : ents->items) {
        if (e.kind != JVal::OBJ) return false;
        PlanEntry pe{};
        if (!as_int(e.get("precision"), 0, 2, &pe.precision) || !as_int(e.get("equation"), 0, 2, &pe.equation) ||
            !as_int(e.get("m_max"), 1, 1 << 20, &pe.m_max) || !as_int(e.get("leaf"), 4, 16, &pe.leaf) ||
            !as_int(e.get("crossover"), -1, 1024, &pe.crossover))
            return false;
        if (pe.leaf != 4 && pe.leaf != 8 && pe.leaf != 16) return false;
        if (pe.crossover == 0) return false;
        got.push_back(pe);
    }
    out.swap(got);
    return true;
}

// Built-in plans, used without a cache file: the tuner's measurements on
// MI355X (gfx950), whole solves of a 4-mode source at N = 16384, gamma = 0.5,
// median of 3 (python -m paper_1710_11593_amd.tune); the comment gives each
// winner's time.  The advection and averaged-spatial-term equations keep the
// plan their kernels were first measured with.
const PlanEntry kBuiltin[] = {
    {0, 0, 64, 16, 512},  // 10.86 ms
    {0, 0, 128, 16, 512},  // 10.86 ms
    {0, 0, 256, 8, 512},  // 13.89 ms
    {0, 0, 512, 8, 256},  // 15.51 ms
    {0, 0, 1024, 8, 128},  // 17.48 ms
    {0, 0, 2048, 8, 128},  // 21.98 ms
    {0, 0, 4096, 8, 128},  // 32.58 ms
    {1, 0, 64, 16, 256},  // 26.76 ms
    {1, 0, 128, 16, 512},  // 27.10 ms
    {1, 0, 256, 8, 256},  // 35.77 ms
    {1, 0, 512, 8, 256},  // 39.82 ms
    {1, 0, 1024, 8, 256},  // 43.46 ms
    {1, 0, 2048, 8, 128},  // 57.31 ms
    {1, 0, 4096, 8, 128},  // 83.46 ms
    {0, 0, 1 << 20, 8, 128},  // 32.58 ms
    {1, 0, 1 << 20, 8, 128},  // 83.46 ms
    {0, 1, 1 << 20, 8, 64},
    {0, 2, 1 << 20, 8, 64},
};

const PlanEntry *lookup(const std::vector<PlanEntry> &tab, int precision, int equation, int64_t mmax)
{
    const PlanEntry *best = nullptr;
    for (const PlanEntry &e : tab)
        if (e.precision == precision && e.equation == equation && mmax <= e.m_max &&
            (!best || e.m_max < best->m_max))
            best = &e;
    return best;
}

}  // namespace

std::string plan_cache_path()
{
    const char *p = getenv("FRACSOLVE_TUNE_CACHE");
    if (p && *p) return p;
    const char *x = getenv("XDG_CACHE_HOME");
    if (x && *x) return std::string(x) + "/fracsolve/plan.json";
    const char *home = getenv("HOME");
    if (home && *home) return std::string(home) + "/.cache/fracsolve/plan.json";
    return std::string();
}

Plan resolve_plan(int precision, int equation, int64_t mmax, int leaf_opt, int crossover_opt)
{
    Plan pl{8, 64, FRACSOLVE_PLAN_BUILTIN};
    const PlanEntry *e = nullptr;
    std::vector<PlanEntry> cache;
    if (leaf_opt == 0 || crossover_opt == 0) {
        const char *t = getenv("FRACSOLVE_TUNE");
        const bool use_cache = !(t && t[0] == '0');
        const std::string path = use_cache ? plan_cache_path() : std::string();
        if (!path.empty() && load_cache(path, cache)) {
            e = lookup(cache, precision, equation, mmax);
            if (e) pl.source = FRACSOLVE_PLAN_CACHE;
        }
        if (!e) {
            std::vector<PlanEntry> tab(kBuiltin, kBuiltin + sizeof kBuiltin / sizeof kBuiltin[0]);
            const PlanEntry *b = lookup(tab, precision, equation, mmax);
            if (b) {
                pl.leaf = b->leaf;
                pl.crossover = b->crossover;
            }
        } else {
            pl.leaf = e->leaf;
            pl.crossover = e->crossover;
        }
    }
    if (leaf_opt != 0) pl.leaf = leaf_opt;
    if (crossover_opt != 0) pl.crossover = crossover_opt;
    if (leaf_opt != 0 && crossover_opt != 0) pl.source = FRACSOLVE_PLAN_OPTIONS;
    return pl;
}

}  // namespace fs
