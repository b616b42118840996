// Launch-shape tuning table: a flat JSON object {"key": integer, ...} written
// by the autotuner (autotune.py next to the library).  Read at context and
// server creation from the path in IRKGL16_TUNE_CACHE, else from
// tune_cache.json beside libirkgl16.so; a missing or unreadable file means the
// built-in defaults.  Only what results do not depend on is tuned: launch
// shapes (systems per workgroup, LDS tile sizes) and the schedule of a call
// (chunk count, promotion and eviction thresholds, keys sched/...).
#include <dlfcn.h>

#include <cctype>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>

#include "launch.h"

namespace irk {

static std::string default_cache_path() {
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&default_cache_path), &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/tune_cache.json";
  }
  return "tune_cache.json";
}

TuneTable load_tune_table() {
  TuneTable t;
  const char* env = std::getenv("IRKGL16_TUNE_CACHE");
  const std::string path = (env && *env) ? std::string(env) : default_cache_path();
  std::ifstream f(path);
  if (!f) return t;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  // "key" : integer pairs; anything else is skipped
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    size_t k = j + 1;
    while (k < s.size() && std::isspace((unsigned char)s[k])) ++k;
    if (k < s.size() && s[k] == ':') {
      ++k;
      while (k < s.size() && std::isspace((unsigned char)s[k])) ++k;
      size_t e = k;
      while (e < s.size() && (std::isdigit((unsigned char)s[e]) || s[e] == '-')) ++e;
      if (e > k) t.values[key] = std::atoi(s.substr(k, e - k).c_str());
      i = e;
    } else {
      i = j + 1;
    }
  }
  return t;
}

int TuneTable::get(const std::string& key, int dflt) const {
  auto it = values.find(key);
  return it == values.end() ? dflt : it->second;
}

std::string wg_tune_key(int kind, int d, int S) {
  return "wg/" + std::to_string(kind) + "/" + std::to_string(d) + "/" + std::to_string(S);
}

std::string large_tune_key(int n) {
  int b = 512;
  while (b < n) b <<= 1;
  return "large/" + std::to_string(b);
}

}  // namespace irk
