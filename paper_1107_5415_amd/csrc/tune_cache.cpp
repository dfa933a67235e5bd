// The batched autotuner's choices, per process and on disk (see tune_cache.hpp).
#include "tune_cache.hpp"

#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace lfft {

namespace {

std::mutex g_mu;
std::map<TuneKey, TuneVal> g_cache;

constexpr const char* kFormat = "lfft-batch-tune";
constexpr int kVersion = 1;

// ---- a small JSON reader: objects, arrays, strings without escapes other
// than \" and \\, numbers kept as their text, true/false/null -------------
struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  std::string text;                                  // NUM: the literal, STR: the value
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* key) const {
    for (const auto& kv : obj)
      if (kv.first == key) return &kv.second;
    return nullptr;
  }
};

struct Parser {
  const char* p;
  const char* end;
  int depth = 0;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool lit(const char* s) {
    const size_t n = std::strlen(s);
    if ((size_t)(end - p) < n || std::strncmp(p, s, n) != 0) return false;
    p += n;
    return true;
  }
  bool str(std::string& out) {
    if (p >= end || *p != '"') return false;
    ++p;
    out.clear();
    while (p < end && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= end || (*p != '"' && *p != '\\')) return false;
      }
      out.push_back(*p++);
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool value(JVal& v) {
    if (++depth > 16) return false;
    ws();
    if (p >= end) return false;
    bool ok = true;
    if (*p == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') {
        ++p;
      } else {
        for (;;) {
          ws();
          std::string k;
          JVal x;
          if (!str(k)) { ok = false; break; }
          ws();
          if (p >= end || *p != ':') { ok = false; break; }
          ++p;
          if (!value(x)) { ok = false; break; }
          v.obj.emplace_back(std::move(k), std::move(x));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == '}') { ++p; break; }
          ok = false;
          break;
        }
      }
    } else if (*p == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') {
        ++p;
      } else {
        for (;;) {
          JVal x;
          if (!value(x)) { ok = false; break; }
          v.arr.push_back(std::move(x));
          ws();
          if (p < end && *p == ',') { ++p; continue; }
          if (p < end && *p == ']') { ++p; break; }
          ok = false;
          break;
        }
      }
    } else if (*p == '"') {
      v.kind = JVal::STR;
      ok = str(v.text);
    } else if (lit("true") || lit("false")) {
      v.kind = JVal::BOOL;
    } else if (lit("null")) {
      v.kind = JVal::NUL;
    } else {
      const char* b = p;
      while (p < end && ((*p != '\0' && std::strchr("+-.eE", *p)) || (*p >= '0' && *p <= '9')))
        ++p;
      v.kind = JVal::NUM;
      v.text.assign(b, p);
      ok = p > b;
    }
    --depth;
    return ok;
  }
};

// integer literal (no fraction or exponent) in [lo, hi]
bool as_int(const JVal* v, long long lo, long long hi, long long& out) {
  if (!v || v->kind != JVal::NUM || v->text.empty()) return false;
  if (v->text.find_first_of(".eE") != std::string::npos) return false;
  errno = 0;
  char* e = nullptr;
  const long long x = std::strtoll(v->text.c_str(), &e, 10);
  if (errno || !e || *e || x < lo || x > hi) return false;
  out = x;
  return true;
}

bool as_num(const JVal* v, double& out) {
  if (!v || v->kind != JVal::NUM) return false;
  char* e = nullptr;
  out = std::strtod(v->text.c_str(), &e);
  return e && !*e;
}

}  // namespace

bool TuneKey::operator<(const TuneKey& o) const {
  if (arch != o.arch) return arch < o.arch;
  if (d != o.d) return d < o.d;
  if (flags != o.flags) return flags < o.flags;
  return Ms < o.Ms;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    throw StatusError{E_HIP};
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

bool tune_cache_find(const TuneKey& k, TuneVal* v) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_cache.find(k);
  if (it == g_cache.end()) return false;
  if (v) *v = it->second;
  return true;
}

void tune_cache_put(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> g(g_mu);
  g_cache[k] = v;
}

void tune_cache_clear() {
  std::lock_guard<std::mutex> g(g_mu);
  g_cache.clear();
}

int tune_cache_size() {
  std::lock_guard<std::mutex> g(g_mu);
  return (int)g_cache.size();
}

void tune_cache_save(const char* path) {
  if (!path || !*path) throw StatusError{E_ARG};
  std::string s;
  {
    std::lock_guard<std::mutex> g(g_mu);
    s = std::string("{\"format\": \"") + kFormat + "\", \"version\": " + std::to_string(kVersion) +
        ", \"entries\": [";
    bool first = true;
    for (const auto& kv : g_cache) {
      const TuneKey& k = kv.first;
      const TuneVal& v = kv.second;
      s += first ? "\n" : ",\n";
      first = false;
      s += "  {\"arch\": \"" + k.arch + "\", \"d\": " + std::to_string(k.d) +
           ", \"flags\": " + std::to_string(k.flags) + ", \"matrices\": [";
      for (size_t i = 0; i < k.Ms.size(); ++i) s += (i ? ", " : "") + std::to_string(k.Ms[i]);
      char ms[32];
      std::snprintf(ms, sizeof ms, "%.6g", (double)v.ms);
      s += "], \"tile_lg\": " + std::to_string(v.tile_lg) + ", \"order\": " +
           std::to_string(v.order) + ", \"ms\": " + ms + "}";
    }
    s += first ? "]}\n" : "\n]}\n";
  }
  FILE* f = std::fopen(path, "wb");
  if (!f) throw StatusError{E_IO};
  const bool ok = std::fwrite(s.data(), 1, s.size(), f) == s.size();
  if (std::fclose(f) != 0 || !ok) throw StatusError{E_IO};
}

int tune_cache_load(const char* path, const std::string& arch) {
  if (!path || !*path) throw StatusError{E_ARG};
  FILE* f = std::fopen(path, "rb");
  if (!f) throw StatusError{E_IO};
  std::string text;
  char buf[65536];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) {
    text.append(buf, n);
    if (text.size() > (size_t(64) << 20)) break;
  }
  const bool rd = !std::ferror(f);
  std::fclose(f);
  if (!rd || text.size() > (size_t(64) << 20)) throw StatusError{E_IO};
  Parser P{text.data(), text.data() + text.size()};
  JVal root;
  if (!P.value(root)) throw StatusError{E_IO};
  P.ws();
  if (P.p != P.end || root.kind != JVal::OBJ) throw StatusError{E_IO};
  const JVal* fmt = root.get("format");
  long long ver = 0;
  if (!fmt || fmt->kind != JVal::STR || fmt->text != kFormat ||
      !as_int(root.get("version"), kVersion, kVersion, ver))
    throw StatusError{E_IO};
  const JVal* ents = root.get("entries");
  if (!ents || ents->kind != JVal::ARR) throw StatusError{E_IO};
  // validate everything before taking anything
  std::vector<std::pair<TuneKey, TuneVal>> take;
  for (const JVal& e : ents->arr) {
    if (e.kind != JVal::OBJ) throw StatusError{E_IO};
    const JVal* a = e.get("arch");
    const JVal* mats = e.get("matrices");
    long long d = 0, flags = 0, tl = 0, ord = 0;
    double ms = -1.0;
    if (!a || a->kind != JVal::STR || !as_int(e.get("d"), 1, 4, d) ||
        !as_int(e.get("flags"), 0, 0xffffffffLL, flags) ||
        !as_int(e.get("tile_lg"), 11, 13, tl) || !as_int(e.get("order"), 0, 7, ord) ||
        !mats || mats->kind != JVal::ARR || mats->arr.empty() ||
        mats->arr.size() % (size_t)(d * d) != 0)
      throw StatusError{E_IO};
    if (e.get("ms") && !as_num(e.get("ms"), ms)) throw StatusError{E_IO};
    TuneKey k;
    k.arch = a->text;
    k.d = (int)d;
    k.flags = (uint32_t)flags;
    for (const JVal& x : mats->arr) {
      long long v = 0;
      if (!as_int(&x, -(1LL << 62), 1LL << 62, v)) throw StatusError{E_IO};
      k.Ms.push_back(v);
    }
    if (k.arch != arch) continue;
    take.push_back({k, TuneVal{(int)tl, (int)ord, (float)ms}});
  }
  std::lock_guard<std::mutex> g(g_mu);
  for (const auto& kv : take) g_cache[kv.first] = kv.second;
  return (int)take.size();
}

}  // namespace lfft
