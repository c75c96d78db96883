// Persisted autotuning: a JSON table of launch configurations keyed by
// device and LP size class.
//
//   {"format": "rgb-tuning-1",
//    "devices": {
//      "<device name> <arch> <CUs>cu": {
//        "variant": "binned", "batched_lanes": 16, "queue_share": 128, "chunk": 1,
//        "grid": 0, "pool_lanes": 4, "pool_wait": 2, "pool_rows": 4, "ms": 1.43,
//        "classes": {"9": {"log2_lanes": 4}, "13": {"log2_lanes": 6}}}}}
//
// A size class c holds the LPs with 2^(c-1) < m <= 2^c rows (the binning of
// the persistent and binned kernels); a class listed in "classes" was tuned
// on a batch in which it held a measurable share of the rows.  Loading
// applies a device's entry on top of the default configuration; saving
// merges: the classes tuned by the latest run replace theirs, the others are
// kept, and the family and its scalar knobs are the latest run's.  Only the
// subset of JSON this file writes is read back (objects, strings, numbers).
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>

#include "rgb_internal.hpp"

namespace rgb {

namespace {

struct JVal {
    enum Kind { kNull, kNum, kStr, kObj } kind = kNull;
    double num = 0.0;
    std::string str;
    std::map<std::string, std::shared_ptr<JVal>> obj;
};

struct Parser {
    const std::string& s;
    size_t i = 0;
    bool ok = true;
    explicit Parser(const std::string& t) : s(t) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    std::string string() {
        std::string out;
        if (!eat('"')) {
            ok = false;
            return out;
        }
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\' && i + 1 < s.size()) ++i;  // the writer never escapes; keep the next byte
            out += s[i++];
        }
        if (i >= s.size()) ok = false;
        ++i;
        return out;
    }
    std::shared_ptr<JVal> value() {
        auto v = std::make_shared<JVal>();
        ws();
        if (i >= s.size()) {
            ok = false;
            return v;
        }
        if (s[i] == '{') {
            ++i;
            v->kind = JVal::kObj;
            if (eat('}')) return v;
            do {
                std::string k = string();
                if (!ok || !eat(':')) {
                    ok = false;
                    return v;
                }
                v->obj[k] = value();
                if (!ok) return v;
            } while (eat(','));
            if (!eat('}')) ok = false;
        } else if (s[i] == '"') {
            v->kind = JVal::kStr;
            v->str = string();
        } else {
            const char* b = s.c_str() + i;
            char* e = nullptr;
            v->num = std::strtod(b, &e);
            if (e == b) {
                ok = false;
                return v;
            }
            v->kind = JVal::kNum;
            i += (size_t)(e - b);
        }
        return v;
    }
};

const char* variant_name(int v) {
    switch (v) {
        case 1: return "plain";
        case 2: return "batched";
        case 3: return "persistent";
        case 4: return "binned";
        case 5: return "pooled";
        default: return "auto";
    }
}

int variant_of(const std::string& n) {
    for (int v = 1; v <= 5; ++v)
        if (n == variant_name(v)) return v;
    return -1;
}

// The whole table; missing file -> empty table (true), unreadable -> false.
bool read_table(const char* path, std::shared_ptr<JVal>& root) {
    root = std::make_shared<JVal>();
    root->kind = JVal::kObj;
    std::ifstream f(path);
    if (!f) return true;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    Parser p(text);
    auto v = p.value();
    if (!p.ok || v->kind != JVal::kObj) return false;
    auto fmt = v->obj.find("format");
    if (fmt == v->obj.end() || fmt->second->kind != JVal::kStr || fmt->second->str != "rgb-tuning-1") return false;
    root = v;
    return true;
}

double num_or(const JVal& o, const char* k, double d) {
    auto it = o.obj.find(k);
    return (it != o.obj.end() && it->second->kind == JVal::kNum) ? it->second->num : d;
}

}  // namespace

int table_load(const char* path, const std::string& device_key, TableEntry& out) {
    std::shared_ptr<JVal> root;
    if (!read_table(path, root)) return -1;
    auto devs = root->obj.find("devices");
    if (devs == root->obj.end() || devs->second->kind != JVal::kObj) return 0;
    auto it = devs->second->obj.find(device_key);
    if (it == devs->second->obj.end() || it->second->kind != JVal::kObj) return 0;
    const JVal& e = *it->second;
    auto var = e.obj.find("variant");
    if (var == e.obj.end() || var->second->kind != JVal::kStr) return -1;
    out.variant = variant_of(var->second->str);
    out.batched_lanes = (int)num_or(e, "batched_lanes", out.batched_lanes);
    out.queue_share = (int)num_or(e, "queue_share", out.queue_share);
    out.chunk = (int)num_or(e, "chunk", out.chunk);
    out.grid = (int)num_or(e, "grid", out.grid);
    out.pool_lanes = (int)num_or(e, "pool_lanes", out.pool_lanes);
    out.pool_wait = (int)num_or(e, "pool_wait", out.pool_wait);
    out.pool_rows = (int)num_or(e, "pool_rows", out.pool_rows);
    out.ms = num_or(e, "ms", 0.0);
    auto cls = e.obj.find("classes");
    if (cls != e.obj.end() && cls->second->kind == JVal::kObj) {
        for (auto& kv : cls->second->obj) {
            char* end = nullptr;
            long c = std::strtol(kv.first.c_str(), &end, 10);
            if (*end || c < 0 || c >= kClasses || kv.second->kind != JVal::kObj) return -1;
            out.log2_lanes[c] = (int)num_or(*kv.second, "log2_lanes", out.log2_lanes[c]);
            out.tuned[c] = true;
        }
    }
    return 1;
}

int table_save(const char* path, const std::string& device_key, const TableEntry& e) {
    std::shared_ptr<JVal> root;
    if (!read_table(path, root)) return -1;
    // classes of this device already in the file and not tuned now are kept
    std::map<int, int> classes;
    auto devs = root->obj.find("devices");
    if (devs != root->obj.end() && devs->second->kind == JVal::kObj) {
        auto it = devs->second->obj.find(device_key);
        if (it != devs->second->obj.end() && it->second->kind == JVal::kObj) {
            auto cls = it->second->obj.find("classes");
            if (cls != it->second->obj.end() && cls->second->kind == JVal::kObj)
                for (auto& kv : cls->second->obj) {
                    int c = std::atoi(kv.first.c_str());
                    if (c >= 0 && c < kClasses && kv.second->kind == JVal::kObj)
                        classes[c] = (int)num_or(*kv.second, "log2_lanes", 2);
                }
        }
    }
    for (int c = 0; c < kClasses; ++c)
        if (e.tuned[c]) classes[c] = e.log2_lanes[c];
    // write every device entry back, this one replaced
    std::ostringstream o;
    o << "{\"format\": \"rgb-tuning-1\",\n \"devices\": {";
    bool first = true;
    auto put_entry = [&](const std::string& key, const TableEntry& t, const std::map<int, int>& cl) {
        o << (first ? "\n" : ",\n") << "  \"" << key << "\": {\"variant\": \"" << variant_name(t.variant)
          << "\", \"batched_lanes\": " << t.batched_lanes << ", \"queue_share\": " << t.queue_share
          << ", \"chunk\": " << t.chunk << ", \"grid\": " << t.grid << ", \"pool_lanes\": " << t.pool_lanes
          << ", \"pool_wait\": " << t.pool_wait << ", \"pool_rows\": " << t.pool_rows << ", \"ms\": " << t.ms
          << ",\n    \"classes\": {";
        bool fc = true;
        for (auto& kv : cl) {
            o << (fc ? "" : ", ") << "\"" << kv.first << "\": {\"log2_lanes\": " << kv.second << "}";
            fc = false;
        }
        o << "}}";
        first = false;
    };
    if (devs != root->obj.end() && devs->second->kind == JVal::kObj)
        for (auto& kv : devs->second->obj) {
            if (kv.first == device_key || kv.second->kind != JVal::kObj) continue;
            TableEntry t;
            if (table_load(path, kv.first, t) != 1) continue;
            std::map<int, int> cl;
            for (int c = 0; c < kClasses; ++c)
                if (t.tuned[c]) cl[c] = t.log2_lanes[c];
            put_entry(kv.first, t, cl);
        }
    put_entry(device_key, e, classes);
    o << "\n }}\n";
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return -1;
        f << o.str();
        if (!f) return -1;
    }
    return std::rename(tmp.c_str(), path) == 0 ? 0 : -1;
}

}  // namespace rgb
