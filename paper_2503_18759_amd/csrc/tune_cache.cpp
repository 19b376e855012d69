// Tuned TTM launch shapes: per-handle table and its JSON file (host only).
#include "tune_cache.h"

#include <hip/hip_runtime.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace cpqr {

namespace {

std::string default_path() {
  const char* env = std::getenv("CPQR_TUNE_CACHE");
  if (env) {
    if (std::strcmp(env, "off") == 0 || env[0] == '\0') return "";
    return env;
  }
  const char* xdg = std::getenv("XDG_CACHE_HOME");
  if (xdg && xdg[0]) return std::string(xdg) + "/cpqr/ttm_tune.json";
  const char* home = std::getenv("HOME");
  if (home && home[0]) return std::string(home) + "/.cache/cpqr/ttm_tune.json";
  return "";
}

// mkdir -p of the directory part of `path`.
bool make_parent_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i) {
    if (path[i] != '/') continue;
    const std::string dir = path.substr(0, i);
    if (::mkdir(dir.c_str(), 0755) != 0 && errno != EEXIST) return false;
  }
  return true;
}

bool read_file(const std::string& path, std::string* text) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  std::ostringstream ss;
  ss << f.rdbuf();
  *text = ss.str();
  return true;
}

// Skips blanks; true if text[*i] == c (consumed).
bool expect(const std::string& t, size_t* i, char c) {
  while (*i < t.size() && (t[*i] == ' ' || t[*i] == '\n' || t[*i] == '\r' || t[*i] == '\t')) ++*i;
  if (*i < t.size() && t[*i] == c) {
    ++*i;
    return true;
  }
  return false;
}

bool read_string(const std::string& t, size_t* i, std::string* out) {
  if (!expect(t, i, '"')) return false;
  const size_t e = t.find('"', *i);
  if (e == std::string::npos) return false;
  *out = t.substr(*i, e - *i);
  *i = e + 1;
  return true;
}

bool read_int(const std::string& t, size_t* i, int* out) {
  while (*i < t.size() && t[*i] == ' ') ++*i;
  size_t j = *i;
  if (j < t.size() && t[j] == '-') ++j;
  if (j >= t.size() || t[j] < '0' || t[j] > '9') return false;
  long v = 0;
  for (; j < t.size() && t[j] >= '0' && t[j] <= '9'; ++j) {
    v = v * 10 + (t[j] - '0');
    if (v > 1000) return false;
  }
  *out = (t[*i] == '-') ? -(int)v : (int)v;
  *i = j;
  return true;
}

bool valid_shape(const TtmShape& s) {
  return (s.ks == 1 || s.ks == 2 || s.ks == 4) && (s.wpc >= 0 && s.wpc <= 2);
}

}  // namespace

std::string tune_cache_format(const std::string& device, const std::map<std::string, TtmShape>& entries) {
  std::ostringstream o;
  o << "{\"format\": 1, \"device\": \"" << device << "\",\n \"entries\": {";
  bool first = true;
  for (const auto& kv : entries) {
    o << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": [" << kv.second.ks << ", " << kv.second.wpc << ']';
    first = false;
  }
  o << "\n }\n}\n";
  return o.str();
}

bool tune_cache_parse(const std::string& t, const std::string& device, std::map<std::string, TtmShape>* entries) {
  size_t i = 0;
  if (!expect(t, &i, '{')) return false;
  std::string dev;
  bool have_dev = false;
  std::map<std::string, TtmShape> got;
  for (;;) {
    std::string name;
    if (!read_string(t, &i, &name) || !expect(t, &i, ':')) return false;
    if (name == "format") {
      int v = 0;
      if (!read_int(t, &i, &v) || v != 1) return false;
    } else if (name == "device") {
      if (!read_string(t, &i, &dev)) return false;
      have_dev = true;
    } else if (name == "entries") {
      if (!expect(t, &i, '{')) return false;
      if (!expect(t, &i, '}')) {
        for (;;) {
          std::string key;
          TtmShape s;
          if (!read_string(t, &i, &key) || !expect(t, &i, ':') || !expect(t, &i, '[') ||
              !read_int(t, &i, &s.ks) || !expect(t, &i, ',') || !read_int(t, &i, &s.wpc) || !expect(t, &i, ']'))
            return false;
          if (key.empty() || key.find('"') != std::string::npos || !valid_shape(s)) return false;
          got[key] = s;
          if (expect(t, &i, ',')) continue;
          if (expect(t, &i, '}')) break;
          return false;
        }
      }
    } else {
      return false;
    }
    if (expect(t, &i, ',')) continue;
    if (expect(t, &i, '}')) break;
    return false;
  }
  if (!have_dev) return false;
  if (dev != device) got.clear();
  *entries = std::move(got);
  return true;
}

TuneCache::TuneCache(int device) : path_(default_path()) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    device_ = std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount);
  } else {
    (void)hipGetLastError();
    device_ = "unknown";
  }
  // a device signature is a plain token inside the file's quotes
  for (char& c : device_)
    if (c == '"' || c == '\\' || c == '\n') c = '_';
}

void TuneCache::load() {
  loaded_ = true;
  if (path_.empty()) return;
  std::string text;
  std::map<std::string, TtmShape> file;
  if (read_file(path_, &text) && tune_cache_parse(text, device_, &file))
    for (const auto& kv : file) mem_.emplace(kv.first, kv.second);
}

bool TuneCache::find(const std::string& key, TtmShape* out) {
  if (!loaded_) load();
  const auto it = mem_.find(key);
  if (it == mem_.end()) return false;
  *out = it->second;
  return true;
}

void TuneCache::put(const std::string& key, const TtmShape& s) {
  if (!loaded_) load();
  mem_[key] = s;
  dirty_ = true;
}

void TuneCache::save() {
  if (!dirty_ || path_.empty()) return;
  dirty_ = false;
  std::map<std::string, TtmShape> merged;
  std::string text;
  if (read_file(path_, &text)) (void)tune_cache_parse(text, device_, &merged);
  for (const auto& kv : mem_) merged[kv.first] = kv.second;
  if (!make_parent_dirs(path_)) return;
  const std::string tmp = path_ + ".tmp." + std::to_string((long)::getpid());
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) return;
    f << tune_cache_format(device_, merged);
    if (!f) {
      f.close();
      (void)std::remove(tmp.c_str());
      return;
    }
  }
  if (std::rename(tmp.c_str(), path_.c_str()) != 0) (void)std::remove(tmp.c_str());
}

std::string ttm_key_single(int prec, int64_t L, int I, int64_t S, int R) {
  return "ttm/p" + std::to_string(prec) + "/L" + std::to_string((long long)L) + "/I" + std::to_string(I) + "/S" +
         std::to_string((long long)S) + "/R" + std::to_string(R);
}

std::string ttm_key_batch(int prec, int nb, bool kc, const std::vector<std::array<int64_t, 4>>& shapes) {
  // FNV-1a over the members' (L, I, S, R)
  uint64_t h = 1469598103934665603ull;
  for (const auto& s : shapes)
    for (int64_t v : s) {
      uint64_t x = (uint64_t)v;
      for (int b = 0; b < 8; ++b) {
        h ^= (x >> (8 * b)) & 0xff;
        h *= 1099511628211ull;
      }
    }
  char hex[17];
  std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)h);
  return "ttmb/p" + std::to_string(prec) + "/nb" + std::to_string(nb) + (kc ? "/kc/" : "/mc/") +
         std::to_string(shapes.size()) + "/" + hex;
}

}  // namespace cpqr
