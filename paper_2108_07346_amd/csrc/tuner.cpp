// The library's tuner: measured choices of launch shapes per device and
// input-shape bucket, kept in memory and, when BR_AUTOTUNE_CACHE names a
// file, in that file (JSON) so that later processes start tuned.
//
// File format: one JSON object whose keys are "<arch>|<path>|<bucket>" and
// whose values are flat objects of numbers, e.g.
//   {"gfx950|plain|v19|e30|m4096": {"solo": 1, "variant": 1, "wpc": 1, ...}}
// Written whole to a temporary file and renamed over the old one.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include <unistd.h>

#include "internal.hpp"

namespace br {

namespace {

struct Cache {
    std::mutex mu;
    bool loaded = false;
    std::string path;
    std::map<std::string, TuneEntry> entries;
};

Cache& cache() {
    static Cache c;
    return c;
}

// minimal reader for the format above (strings without escapes, numbers)
struct Reader {
    const std::string& s;
    size_t i = 0;
    void ws() { while (i < s.size() && std::isspace((unsigned char)s[i])) i++; }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) { i++; return true; }
        return false;
    }
    bool str(std::string& out) {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        size_t j = s.find('"', i + 1);
        if (j == std::string::npos) return false;
        out = s.substr(i + 1, j - i - 1);
        i = j + 1;
        return true;
    }
    bool num(double& out) {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        out = std::strtod(b, &e);
        if (e == b) return false;
        i += (size_t)(e - b);
        return true;
    }
};

bool parse(const std::string& text, std::map<std::string, TuneEntry>& out) {
    Reader r{text};
    if (!r.eat('{')) return false;
    if (r.eat('}')) return true;
    do {
        std::string key;
        if (!r.str(key) || !r.eat(':') || !r.eat('{')) return false;
        TuneEntry e;
        if (!r.eat('}')) {
            do {
                std::string f;
                double v = 0;
                if (!r.str(f) || !r.eat(':') || !r.num(v)) return false;
                e[f] = v;
            } while (r.eat(','));
            if (!r.eat('}')) return false;
        }
        out[key] = e;
    } while (r.eat(','));
    return r.eat('}');
}

std::string to_json(const std::map<std::string, TuneEntry>& m) {
    std::ostringstream o;
    o << "{\n";
    bool first = true;
    for (const auto& kv : m) {
        o << (first ? "" : ",\n") << " \"" << kv.first << "\": {";
        first = false;
        bool f2 = true;
        for (const auto& fv : kv.second) {
            char buf[64];
            std::snprintf(buf, sizeof buf, "%.6g", fv.second);
            o << (f2 ? "" : ", ") << "\"" << fv.first << "\": " << buf;
            f2 = false;
        }
        o << "}";
    }
    o << "\n}\n";
    return o.str();
}

void load_locked(Cache& c) {
    if (c.loaded) return;
    c.loaded = true;
    const char* p = std::getenv("BR_AUTOTUNE_CACHE");
    if (!p || !*p) return;
    c.path = p;
    std::ifstream f(c.path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    std::map<std::string, TuneEntry> m;
    if (parse(ss.str(), m)) c.entries = m;   // an unreadable file is ignored (and rewritten on the next save)
}

}  // namespace

std::string arch_name(int device) {
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> g(mu);
    auto it = names.find(device);
    if (it != names.end()) return it->second;
    hipDeviceProp_t p;
    std::string n = "unknown";
    if (hipGetDeviceProperties(&p, device) == hipSuccess) {
        n = p.gcnArchName;
        const size_t colon = n.find(':');   // drop feature suffixes (":sramecc+:xnack-")
        if (colon != std::string::npos) n = n.substr(0, colon);
    } else {
        (void)hipGetLastError();
    }
    names[device] = n;
    return n;
}

int log2_bucket(int64_t x) {
    int b = 0;
    while ((int64_t(1) << b) < x && b < 62) b++;
    return b;
}

bool tune_get(const std::string& key, TuneEntry& out) {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    load_locked(c);
    auto it = c.entries.find(key);
    if (it == c.entries.end()) return false;
    out = it->second;
    return true;
}

void tune_put(const std::string& key, const TuneEntry& e) {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    load_locked(c);
    c.entries[key] = e;
    if (c.path.empty()) return;
    // merge with what other processes wrote meanwhile, then replace the file
    std::map<std::string, TuneEntry> disk;
    {
        std::ifstream f(c.path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            if (parse(ss.str(), disk))
                for (const auto& kv : disk)
                    if (!c.entries.count(kv.first)) c.entries[kv.first] = kv.second;
        }
    }
    const std::string tmp = c.path + ".tmp" + std::to_string((long long)getpid());
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return;
        f << to_json(c.entries);
    }
    std::rename(tmp.c_str(), c.path.c_str());
}

}  // namespace br
