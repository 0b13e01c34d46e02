// Sanitizer driver for the plan-cache reader of the library (test
// infrastructure): paper_1710_11593_amd/csrc/plan.hip is pure host C++ and
// is compiled here with g++ and -fsanitize=address,undefined by
// tests/test_sanitize_host.py.  It feeds resolve_plan well-formed caches,
// hand-made malformed ones and a few thousand seeded mutations of a valid
// file, and checks that every result is a plan the library can run (leaf 4,
// 8 or 16; crossover -1 or 1..1024; explicit options always win).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/fracsolve.h"
#include "../../paper_1710_11593_amd/csrc/plan.hpp"

static int fails = 0;

static void write(const std::string &path, const std::string &text)
{
    FILE *f = fopen(path.c_str(), "wb");
    if (!f) {
        perror("fopen");
        exit(2);
    }
    fwrite(text.data(), 1, text.size(), f);
    fclose(f);
}

static void check(const fs::Plan &p, const char *what)
{
    const bool leaf_ok = p.leaf == 4 || p.leaf == 8 || p.leaf == 16;
    const bool cross_ok = p.crossover == -1 || (p.crossover >= 1 && p.crossover <= 1024);
    if (!leaf_ok || !cross_ok) {
        fprintf(stderr, "%s: plan leaf %d crossover %d source %d\n", what, p.leaf, p.crossover, p.source);
        ++fails;
    }
}

int main(int argc, char **argv)
{
    const std::string path = std::string(argc > 1 ? argv[1] : "/tmp") + "/plan.json";
    setenv("FRACSOLVE_TUNE_CACHE", path.c_str(), 1);
    unsetenv("FRACSOLVE_TUNE");
    const std::string valid =
        "{\"fracsolve_plan\": 1, \"device\": \"gfx950\", \"entries\": ["
        "{\"precision\": 0, \"equation\": 0, \"m_max\": 256, \"leaf\": 16, \"crossover\": 512},"
        "{\"precision\": 0, \"equation\": 0, \"m_max\": 4096, \"leaf\": 8, \"crossover\": 128},"
        "{\"precision\": 1, \"equation\": 0, \"m_max\": 1048576, \"leaf\": 4, \"crossover\": -1}]}";
    write(path, valid);
    fs::Plan p = fs::resolve_plan(0, 0, 100, 0, 0);
    if (p.leaf != 16 || p.crossover != 512 || p.source != FRACSOLVE_PLAN_CACHE) ++fails;
    p = fs::resolve_plan(1, 0, 5000, 0, 0);
    if (p.leaf != 4 || p.crossover != -1) ++fails;
    p = fs::resolve_plan(0, 2, 100, 0, 0);  // no entry for this equation
    if (p.source != FRACSOLVE_PLAN_BUILTIN) ++fails;
    check(p, "builtin");
    const char *bad[] = {
        "", "{", "}", "[]", "null", "\"x\"", "{\"fracsolve_plan\": 1}", "{\"fracsolve_plan\": 1, \"entries\": 5}",
        "{\"fracsolve_plan\": 1, \"entries\": [1, 2]}", "{\"fracsolve_plan\": 1e400, \"entries\": []}",
        "{\"fracsolve_plan\": 1, \"entries\": [{\"precision\": -0, \"equation\": 0, \"m_max\": 9e18, "
        "\"leaf\": 8, \"crossover\": 64}]}",
        "{\"a\\", "{\"a\\u0041\": 1}", "{\"fracsolve_plan\": 1, \"entries\": [{\"leaf\": nan}]}",
        "{\"fracsolve_plan\": 1, \"entries\": [{\"precision\": 0, \"equation\": 0, \"m_max\": 64, \"leaf\": 8, "
        "\"crossover\": 64},]}",
    };
    for (const char *b : bad) {
        write(path, b);
        for (int prec = 0; prec < 2; ++prec) check(fs::resolve_plan(prec, 0, 300, 0, 0), b);
    }
    // nesting far deeper than the reader's limit
    write(path, std::string(100000, '[') + std::string(100000, ']'));
    check(fs::resolve_plan(0, 0, 300, 0, 0), "deep nesting");
    write(path, "{\"k\": " + std::string(50000, '[') + "}");
    check(fs::resolve_plan(0, 0, 300, 0, 0), "deep unclosed nesting");
    // seeded mutations of the valid file: flips, deletions, insertions, truncations
    unsigned seed = 12345u;
    auto rnd = [&](unsigned n) {
        seed = seed * 1103515245u + 12345u;
        return (seed >> 8) % n;
    };
    const char alphabet[] = "{}[]\":,.-+eE0123456789 \\tnrufalse";
    for (int it = 0; it < 4000; ++it) {
        std::string t = valid;
        const int edits = 1 + (int)rnd(4);
        for (int e = 0; e < edits && !t.empty(); ++e) {
            const size_t at = rnd((unsigned)t.size());
            switch (rnd(4)) {
                case 0: t[at] = alphabet[rnd(sizeof alphabet - 1)]; break;
                case 1: t.erase(at, 1 + rnd(8)); break;
                case 2: t.insert(at, 1, alphabet[rnd(sizeof alphabet - 1)]); break;
                default: t.resize(at); break;
            }
        }
        write(path, t);
        for (int prec = 0; prec < 2; ++prec)
            for (int64_t m : {1, 257, 4096, 1 << 20}) {
                check(fs::resolve_plan(prec, 0, m, 0, 0), "mutation");
                const fs::Plan o = fs::resolve_plan(prec, 0, m, 4, 32);
                if (o.leaf != 4 || o.crossover != 32 || o.source != FRACSOLVE_PLAN_OPTIONS) ++fails;
            }
    }
    // a missing file and FRACSOLVE_TUNE=0
    remove(path.c_str());
    check(fs::resolve_plan(0, 0, 300, 0, 0), "missing file");
    setenv("FRACSOLVE_TUNE", "0", 1);
    write(path, valid);
    if (fs::resolve_plan(0, 0, 100, 0, 0).source != FRACSOLVE_PLAN_BUILTIN) ++fails;
    if (fails) {
        fprintf(stderr, "%d failures\n", fails);
        return 1;
    }
    printf("plan driver: all cases clean\n");
    return 0;
}
