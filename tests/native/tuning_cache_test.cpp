// Host-only checks of the schedule autotuner's tuning-cache file
// (csrc/tuning_cache.hpp), built with AddressSanitizer and UBSan by
// tests/test_native_tuning_cache.py: round trips, every truncation and
// single-byte corruption of a valid file parse or fail cleanly, malformed
// files are refused.
#include <cstdio>
#include <cstring>
#include <string>

#include "tuning_cache.hpp"

using slaq::tuning::Entries;
using slaq::tuning::parse_cache;

static int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "%s:%d: CHECK(%s)\n", __FILE__, __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    const std::string path = dir + "/cache.json";
    Entries e;
    e["gfx950:sramecc+:xnack-|lap0-prec0-rel1-ld100-n26-nnz31"] = {
        {"heavy_min", 256}, {"piece", 256}, {"cache_rows", -1}, {"fused", -1}, {"ms", 525.7294921875}};
    e["odd \"key\" \\ with escapes"] = {{"x", 1e-300}, {"y", -2.5e17}};
    e["empty"] = {};
    CHECK(slaq::tuning::write_cache(path.c_str(), e));
    std::string text;
    CHECK(slaq::tuning::read_file(path.c_str(), text));
    Entries back;
    CHECK(parse_cache(text, back));
    CHECK(back == e);

    // every prefix that stops short of the closing brace is refused
    const size_t last = text.find_last_of('}');
    for (size_t k = 0; k <= last; ++k) {
        Entries x;
        CHECK(!parse_cache(text.substr(0, k), x));
    }
    // every single-byte corruption parses or fails without touching memory out of bounds
    const char subs[] = {'{', '}', '"', ':', ',', '\\', '0', 'e', '-', ' ', '\0'};
    for (size_t k = 0; k < text.size(); ++k)
        for (char c : subs) {
            std::string t = text;
            t[k] = c;
            Entries x;
            (void)parse_cache(t.c_str(), x);  // stops at an embedded NUL like the library
        }
    const char* bad[] = {"", "[]", "{", "{}}", "{\"a\": 1}", "{\"a\": {\"b\": }}", "{\"a\": {\"b\": 1,}}",
                         "{\"a\" {\"b\": 1}}", "{\"a\": {\"b\": 1}} trailing", "{\"a\": {\"b\": \"s\"}}",
                         "{\"unterminated: {}}"};
    for (const char* b : bad) {
        Entries x;
        CHECK(!parse_cache(b, x));
    }
    Entries x;
    CHECK(parse_cache("  {}  \n", x) && x.empty());
    CHECK(parse_cache("{\"k\": {\"a\": -1.5e-3, \"b\": 7}}", x) && x["k"]["a"] == -1.5e-3 && x["k"]["b"] == 7);
    CHECK(!slaq::tuning::read_file((dir + "/missing.json").c_str(), text));
    std::printf("%s (%d failures)\n", failures ? "FAIL" : "ok", failures);
    return failures ? 1 : 0;
}
