// Autotuner: picks the engine's tuning knobs (radix digit width, fused or
// separate difference pass, tuple-set and index load factors, grid cap of the
// look-back kernels, block size of the join and difference kernels per launch
// size bucket) by timed trials on the caller's own workload, and keeps
// the winners in a small JSON cache keyed by GPU architecture and a caller
// key.  The knobs change speed and memory only; every trial computes the same
// fixpoint.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fv.h"

namespace fv {
std::string& global_error() {   // error text of calls that have no context
  static std::string e;
  return e;
}
}  // namespace fv

namespace {

#define g_error (fv::global_error())

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// --- a minimal reader/writer for {"entries": {"<arch>/<key>": {"knob": number, ...}}}
using Entry = std::map<std::string, double>;

bool parse_cache(const std::string& text, std::map<std::string, Entry>& out) {
  size_t p = text.find("\"entries\"");
  if (p == std::string::npos) return false;
  p = text.find('{', p);
  if (p == std::string::npos) return false;
  ++p;
  auto skip = [&]() { while (p < text.size() && std::isspace(static_cast<unsigned char>(text[p]))) ++p; };
  auto str = [&](std::string& s) {
    skip();
    if (p >= text.size() || text[p] != '"') return false;
    const size_t e = text.find('"', p + 1);
    if (e == std::string::npos) return false;
    s = text.substr(p + 1, e - p - 1);
    p = e + 1;
    return true;
  };
  for (;;) {
    skip();
    if (p >= text.size()) return false;
    if (text[p] == '}') return true;
    if (text[p] == ',') { ++p; continue; }
    std::string name;
    if (!str(name)) return false;
    skip();
    if (p >= text.size() || text[p] != ':') return false;
    ++p;
    skip();
    if (p >= text.size() || text[p] != '{') return false;
    ++p;
    Entry e;
    for (;;) {
      skip();
      if (p >= text.size()) return false;
      if (text[p] == '}') { ++p; break; }
      if (text[p] == ',') { ++p; continue; }
      std::string k;
      if (!str(k)) return false;
      skip();
      if (p >= text.size() || text[p] != ':') return false;
      ++p;
      char* end = nullptr;
      const double v = std::strtod(text.c_str() + p, &end);
      if (end == text.c_str() + p) return false;
      p = size_t(end - text.c_str());
      e[k] = v;
    }
    out[name] = e;
  }
}

std::string render_cache(const std::map<std::string, Entry>& entries) {
  std::ostringstream o;
  o << "{\n \"format\": \"fv-tuning-1\",\n \"entries\": {";
  bool first = true;
  for (auto& kv : entries) {
    o << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": {";
    bool f2 = true;
    for (auto& kv2 : kv.second) {
      char buf[64];
      std::snprintf(buf, sizeof(buf), "%.6g", kv2.second);
      o << (f2 ? "" : ", ") << "\"" << kv2.first << "\": " << buf;
      f2 = false;
    }
    o << "}";
    first = false;
  }
  o << "\n }\n}\n";
  return o.str();
}

// block_log2[c][b] is stored as "block_<class>_b<bucket>"
const char* const kBlockClass[2] = {"join", "dedup"};

std::string block_key(int c, int b) { return std::string("block_") + kBlockClass[c] + "_b" + std::to_string(b); }

Entry to_entry(const fv_tuning& t, double ms) {
  Entry e{{"radix_bits", double(t.radix_bits)}, {"fuse_dedup", double(t.fuse_dedup)},
          {"set_load", double(t.set_load)},     {"index_load", double(t.index_load)},
          {"max_blocks", double(t.max_blocks)}, {"index_rebuild", double(t.index_rebuild)},
          {"index_sort", double(t.index_sort)},   {"lookahead", double(t.lookahead)},
          {"dedup_ranges", double(t.dedup_ranges)}, {"ms", ms}};
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 4; ++b) e[block_key(c, b)] = t.block_log2[c][b] ? t.block_log2[c][b] : 8;
  return e;
}

fv_tuning from_entry(const Entry& e) {
  fv_tuning t{};
  auto get = [&](const char* k, double d) { auto it = e.find(k); return it == e.end() ? d : it->second; };
  t.radix_bits = uint32_t(get("radix_bits", 8));
  t.fuse_dedup = uint32_t(get("fuse_dedup", 0));
  t.set_load = float(get("set_load", 0.25));
  t.index_load = float(get("index_load", 0.5));
  t.max_blocks = uint32_t(get("max_blocks", 2048));
  t.index_rebuild = uint32_t(get("index_rebuild", 0));
  t.index_sort = uint32_t(get("index_sort", 0));
  t.lookahead = uint32_t(get("lookahead", 0));
  t.dedup_ranges = uint32_t(get("dedup_ranges", 0));
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 4; ++b) t.block_log2[c][b] = uint8_t(get(block_key(c, b).c_str(), 8));
  return t;
}

// Median fv_run_fixpoint time (ms) of `reps` fresh contexts with tuning t,
// or a negative value if a trial failed.
double trial(fv_make_ctx_fn make, void* user, const fv_options* base, const fv_tuning& t, uint32_t reps) {
  fv_options opt = base ? *base : fv_options{};
  opt.tuning = &t;
  std::vector<double> ms;
  for (uint32_t r = 0; r < reps; ++r) {
    fv_ctx* ctx = make(&opt, user);
    if (!ctx) { g_error = "the context factory returned NULL"; return -1; }
    fv_stats st{};
    const fv_status rc = fv_run_fixpoint(ctx, &st);
    if (rc != FV_OK) {
      g_error = std::string("trial failed: ") + fv_last_error(ctx);
      fv_ctx_destroy(ctx);
      return -1;
    }
    ms.push_back(st.ms_total);
    fv_ctx_destroy(ctx);
  }
  std::sort(ms.begin(), ms.end());
  return ms[ms.size() / 2];
}

}  // namespace

extern "C" {

const char* fv_global_error(void) { return g_error.c_str(); }

fv_status fv_tuning_load(const char* cache_path, const char* key, fv_tuning* out) {
  if (!cache_path || !key || !out) return FV_EINVAL;
  std::ifstream f(cache_path);
  if (!f) { g_error = "cannot open tuning cache"; return FV_EINVAL; }
  std::stringstream ss;
  ss << f.rdbuf();
  std::map<std::string, Entry> entries;
  if (!parse_cache(ss.str(), entries)) { g_error = "malformed tuning cache"; return FV_EINVAL; }
  auto it = entries.find(device_arch() + "/" + key);
  if (it == entries.end()) { g_error = "no tuning stored for this key and GPU"; return FV_EINVAL; }
  *out = from_entry(it->second);
  return FV_OK;
}

fv_status fv_autotune(fv_make_ctx_fn make, void* user, const fv_options* base, uint32_t reps,
                      const char* cache_path, const char* key, fv_tuning* best) {
  if (!make || !best) return FV_EINVAL;
  if (reps == 0) reps = 3;
  fv_tuning cur{};
  cur.radix_bits = 8;
  cur.fuse_dedup = 0;
  cur.set_load = 0.25f;
  cur.index_load = 0.5f;
  cur.max_blocks = 2048;
  for (auto& cls : cur.block_log2)
    for (auto& l : cls) l = 8;
  double cur_ms = trial(make, user, base, cur, reps);
  if (cur_ms < 0) return FV_EINVAL;
  // coordinate search: each knob in turn, the others at their best so far
  const std::vector<double> radix = {8, 11}, fuse = {0, 1}, sload = {0.25, 0.5}, iload = {0.25, 0.5},
                            blocks = {1024, 2048, 4096}, rebuild = {0, 1},
                            isort = {0, 1}, ahead = {0, 1}, block = {7, 8, 9},
                            // (Algorithm 2's difference, mode 1, is left out: on skewed data one
                            // trial can take a hundred times the others)
                            ranges = {0, 2};
  struct Knob { const std::vector<double>* vals; int which; };
  // then the block size of each kernel class in each launch size bucket
  // (a bucket no launch falls in times the same as the default and keeps it)
  std::vector<Knob> knobs = {{&radix, 0}, {&fuse, 1}, {&sload, 2}, {&iload, 3}, {&blocks, 4}, {&rebuild, 5},
                             {&isort, 6}, {&ahead, 7}, {&ranges, 8}};
  for (int w = 100; w < 108; ++w) knobs.push_back({&block, w});
  for (const Knob& k : knobs) {
    for (double v : *k.vals) {
      fv_tuning t = cur;
      switch (k.which) {
        case 0: t.radix_bits = uint32_t(v); break;
        case 1: t.fuse_dedup = uint32_t(v); break;
        case 2: t.set_load = float(v); break;
        case 3: t.index_load = float(v); break;
        case 4: t.max_blocks = uint32_t(v); break;
        case 5: t.index_rebuild = uint32_t(v); break;
        case 6: t.index_sort = uint32_t(v); break;
        case 7: t.lookahead = uint32_t(v); break;
        case 8: t.dedup_ranges = uint32_t(v); break;
        default: t.block_log2[(k.which - 100) / 4][(k.which - 100) % 4] = uint8_t(v); break;
      }
      if (std::memcmp(&t, &cur, sizeof(t)) == 0) continue;
      // a candidate whose trial fails (out of memory, say) is passed over;
      // only the defaults' trial must succeed
      const double ms = trial(make, user, base, t, reps);
      if (ms >= 0 && ms < cur_ms) { cur = t; cur_ms = ms; }
    }
  }
  *best = cur;
  if (cache_path && key) {
    std::map<std::string, Entry> entries;
    {
      std::ifstream f(cache_path);
      if (f) {
        std::stringstream ss;
        ss << f.rdbuf();
        parse_cache(ss.str(), entries);
      }
    }
    entries[device_arch() + "/" + key] = to_entry(cur, cur_ms);
    std::ofstream o(cache_path);
    if (!o) { g_error = "cannot write tuning cache"; return FV_EINVAL; }
    o << render_cache(entries);
  }
  return FV_OK;
}

}  // extern "C"
