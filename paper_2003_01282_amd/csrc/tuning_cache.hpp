// Tuning cache file of the schedule autotuner: a flat JSON object whose
// values are objects of numeric fields,
//   {"<key>": {"<field>": <number>, ...}, ...}
// read and written whole.  Plain host C++ (no HIP), so that a host-only test
// program can exercise it under AddressSanitizer / UBSan.
#pragma once

#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

namespace slaq {
namespace tuning {

using Entries = std::map<std::string, std::map<std::string, double>>;

inline void skip_ws(const char*& s) {
    while (*s == ' ' || *s == '\n' || *s == '\r' || *s == '\t') ++s;
}

inline bool parse_string(const char*& s, std::string& out) {
    skip_ws(s);
    if (*s != '"') return false;
    ++s;
    out.clear();
    while (*s && *s != '"') {
        if (*s == '\\' && s[1]) ++s;
        out.push_back(*s++);
    }
    if (*s != '"') return false;
    ++s;
    return true;
}

inline bool expect(const char*& s, char c) {
    skip_ws(s);
    if (*s != c) return false;
    ++s;
    return true;
}

// false on anything that is not such an object (out may then hold a prefix)
inline bool parse_cache(const std::string& text, Entries& out) {
    const char* s = text.c_str();
    if (!expect(s, '{')) return false;
    skip_ws(s);
    if (*s == '}') {
        ++s;
        skip_ws(s);
        return *s == 0;
    }
    for (;;) {
        std::string key;
        if (!parse_string(s, key) || !expect(s, ':') || !expect(s, '{')) return false;
        std::map<std::string, double> fields;
        skip_ws(s);
        if (*s != '}') {
            for (;;) {
                std::string name;
                if (!parse_string(s, name) || !expect(s, ':')) return false;
                skip_ws(s);
                char* end = nullptr;
                const double v = std::strtod(s, &end);
                if (end == s) return false;
                s = end;
                fields[name] = v;
                skip_ws(s);
                if (*s == ',') {
                    ++s;
                    continue;
                }
                break;
            }
        }
        if (!expect(s, '}')) return false;
        out[key] = fields;
        skip_ws(s);
        if (*s == ',') {
            ++s;
            continue;
        }
        break;
    }
    if (!expect(s, '}')) return false;
    skip_ws(s);
    return *s == 0;  // nothing after the object
}

inline bool read_file(const char* path, std::string& text) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t k;
    text.clear();
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    std::fclose(f);
    return true;
}

// JSON string body of s (quotes and backslashes escaped)
inline std::string quoted(const std::string& s) {
    std::string o = "\"";
    for (char c : s) {
        if (c == '"' || c == '\\') o.push_back('\\');
        o.push_back(c);
    }
    o.push_back('"');
    return o;
}

// written to path.tmp, then renamed over path
inline bool write_cache(const char* path, const Entries& entries) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{");
    bool first = true;
    for (const auto& e : entries) {
        std::fprintf(f, "%s\n %s: {", first ? "" : ",", quoted(e.first).c_str());
        bool ff = true;
        for (const auto& kv : e.second) {
            std::fprintf(f, "%s%s: %.17g", ff ? "" : ", ", quoted(kv.first).c_str(), kv.second);
            ff = false;
        }
        std::fprintf(f, "}");
        first = false;
    }
    std::fprintf(f, "\n}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace tuning
}  // namespace slaq
