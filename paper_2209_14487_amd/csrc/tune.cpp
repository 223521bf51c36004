// The tile cache of cq_crowd_autotune_tiles: a JSON array with one flat object per line,
// keyed by device, N, walkers, precision and delay rank.  Host code only; the reader takes
// the file as this writer makes it (one object per line, string values without escapes,
// numbers) and skips any line that does not parse.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "cq.h"
#include "cq_host.h"

namespace {

bool valid_device(const char* d)
{
    if (!d || !*d || std::strlen(d) > 127) return false;
    for (const char* p = d; *p; ++p)
        if (*p == '"' || *p == '\\' || (unsigned char)*p < 0x20) return false;
    return true;
}

const char* prec_name(int p) { return p == CQ_FP64 ? "fp64" : "mixed"; }

// {"key": "str" | number, ...} on one line (a trailing comma allowed) -> key -> raw value
bool parse_line(const std::string& line, std::map<std::string, std::string>& out)
{
    size_t i = line.find_first_not_of(" \t\r");
    if (i == std::string::npos || line[i] != '{') return false;
    size_t end = line.find_last_not_of(" \t\r,");
    if (end == std::string::npos || line[end] != '}' || end <= i) return false;
    ++i;
    while (i < end) {
        i = line.find_first_not_of(" \t", i);
        if (i >= end) break;
        if (line[i] != '"') return false;
        const size_t k1 = line.find('"', i + 1);
        if (k1 == std::string::npos || k1 >= end) return false;
        const std::string key = line.substr(i + 1, k1 - i - 1);
        i = line.find_first_not_of(" \t", k1 + 1);
        if (i >= end || line[i] != ':') return false;
        i = line.find_first_not_of(" \t", i + 1);
        if (i >= end) return false;
        std::string val;
        if (line[i] == '"') {
            const size_t v1 = line.find('"', i + 1);
            if (v1 == std::string::npos || v1 >= end) return false;
            val = line.substr(i + 1, v1 - i - 1);
            i = v1 + 1;
        } else {
            size_t v1 = i;
            while (v1 < end && line[v1] != ',' && line[v1] != ' ' && line[v1] != '\t') ++v1;
            val = line.substr(i, v1 - i);
            if (val.empty()) return false;
            char* stop = nullptr;
            (void)std::strtod(val.c_str(), &stop);
            if (!stop || *stop) return false;
            i = v1;
        }
        out[key] = val;
        i = line.find_first_not_of(" \t", i);
        if (i < end) {
            if (line[i] != ',') return false;
            ++i;
        }
    }
    return true;
}

bool get_int(const std::map<std::string, std::string>& m, const char* key, long* v)
{
    auto it = m.find(key);
    if (it == m.end()) return false;
    char* stop = nullptr;
    const long x = std::strtol(it->second.c_str(), &stop, 10);
    if (!stop || *stop) return false;
    *v = x;
    return true;
}

bool read_lines(const char* path, std::vector<std::string>& lines, bool* exists)
{
    FILE* f = std::fopen(path, "r");
    *exists = f != nullptr;
    if (!f) return errno == ENOENT;
    std::string cur;
    int ch;
    while ((ch = std::fgetc(f)) != EOF) {
        if (ch == '\n') {
            lines.push_back(cur);
            cur.clear();
        } else {
            cur.push_back((char)ch);
        }
    }
    if (!cur.empty()) lines.push_back(cur);
    const bool ok = !std::ferror(f);
    std::fclose(f);
    return ok;
}

bool matches(const std::map<std::string, std::string>& m, const char* device, int n, int walkers, int precision,
             int delay_rank)
{
    auto d = m.find("device");
    auto p = m.find("precision");
    long vn, vw, vk;
    return d != m.end() && d->second == device && p != m.end() && p->second == prec_name(precision) &&
           get_int(m, "n", &vn) && vn == n && get_int(m, "walkers", &vw) && vw == walkers &&
           get_int(m, "delay_rank", &vk) && vk == delay_rank;
}

}  // namespace

extern "C" cq_status cq_tile_cache_find(const char* path, const char* device, int n, int walkers, int precision,
                                        int delay_rank, cq_tiles* out, int* found)
{
    if (!path || !out || !found) return cq::host_fail(CQ_EINVAL, "tile cache: NULL argument");
    if (!valid_device(device)) return cq::host_fail(CQ_EINVAL, "tile cache: bad device name");
    if (n < 1 || walkers < 1 || delay_rank < 1 || (precision != CQ_FP64 && precision != CQ_MIXED))
        return cq::host_fail(CQ_EINVAL, "tile cache: bad key");
    *found = 0;
    std::vector<std::string> lines;
    bool exists = false;
    if (!read_lines(path, lines, &exists)) return cq::host_fail(CQ_EIO, std::string("tile cache: cannot read ") + path);
    for (const std::string& line : lines) {
        std::map<std::string, std::string> m;
        long q, g;
        if (!parse_line(line, m) || !matches(m, device, n, walkers, precision, delay_rank)) continue;
        if (!get_int(m, "candidates", &q) || !get_int(m, "gather_blocks_per_cu", &g)) continue;
        long u = 0;
        if (m.count("update_kernel") && !get_int(m, "update_kernel", &u)) continue;
        if (q < 0 || q > 1 << 20 || g < 0 || g > 64 || u < 0 || u > 2) continue;
        out->candidates = (int)q;
        out->gather_blocks_per_cu = (int)g;
        out->update_kernel = (int)u;
        *found = 1;  // keep scanning: the last matching entry wins
    }
    return CQ_OK;
}

extern "C" cq_status cq_tile_cache_store(const char* path, const char* device, int n, int walkers, int precision,
                                         int delay_rank, const cq_tiles* t, double ms_per_sweep)
{
    if (!path || !t) return cq::host_fail(CQ_EINVAL, "tile cache: NULL argument");
    if (!valid_device(device)) return cq::host_fail(CQ_EINVAL, "tile cache: bad device name");
    if (n < 1 || walkers < 1 || delay_rank < 1 || (precision != CQ_FP64 && precision != CQ_MIXED) ||
        t->candidates < 0 || t->gather_blocks_per_cu < 0 || t->gather_blocks_per_cu > 64 || t->update_kernel < 0 ||
        t->update_kernel > 2 || !(ms_per_sweep >= 0.0))
        return cq::host_fail(CQ_EINVAL, "tile cache: bad entry");
    std::vector<std::string> lines;
    bool exists = false;
    if (!read_lines(path, lines, &exists)) return cq::host_fail(CQ_EIO, std::string("tile cache: cannot read ") + path);
    std::vector<std::string> keep;
    for (std::string& line : lines) {
        std::map<std::string, std::string> m;
        if (!parse_line(line, m)) continue;
        const size_t end = line.find_last_not_of(" \t\r,");
        keep.push_back(line.substr(line.find_first_not_of(" \t\r"), end + 1 - line.find_first_not_of(" \t\r")));
    }
    char buf[512];
    std::snprintf(buf, sizeof buf,
                  "{\"device\": \"%s\", \"n\": %d, \"walkers\": %d, \"precision\": \"%s\", \"delay_rank\": %d, "
                  "\"candidates\": %d, \"gather_blocks_per_cu\": %d, \"update_kernel\": %d, \"ms_per_sweep\": %.6g}",
                  device, n, walkers, prec_name(precision), delay_rank, t->candidates, t->gather_blocks_per_cu,
                  t->update_kernel, ms_per_sweep);
    keep.push_back(buf);
    // write a sibling file, then rename it over the cache
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return cq::host_fail(CQ_EIO, std::string("tile cache: cannot write ") + tmp);
    bool ok = std::fputs("[\n", f) >= 0;
    for (size_t i = 0; ok && i < keep.size(); ++i)
        ok = std::fputs(keep[i].c_str(), f) >= 0 && std::fputs(i + 1 < keep.size() ? ",\n" : "\n", f) >= 0;
    ok = ok && std::fputs("]\n", f) >= 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return cq::host_fail(CQ_EIO, std::string("tile cache: cannot write ") + path);
    }
    return CQ_OK;
}
