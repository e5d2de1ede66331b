// Tile-shape cache of the autotuner: a JSON file holding one object,
//   { "<key>": {"cfg": <tile shape>, "box": <box shape>, "ms": <mean time per apply>}, ... }
// with keys naming the operator (kind, precision, boundary condition, rule,
// level, macros, map) or the batch (kind, precision, the instances' levels and
// macro counts) and the device (architecture, compute units); cfg is the
// fastest shape, box the fastest box shape (used by the modes the marching
// shapes do not provide).  A tuned shape is looked up before timing; a new
// result is merged into the file, which is rewritten through a temporary file
// and a rename.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

#include "host_internal.h"

namespace {

struct Entry {
  int cfg = 0, box = 0;
  double ms = 0.0;
};

void skip_ws(const std::string &t, size_t &i) {
  while (i < t.size() && std::isspace(static_cast<unsigned char>(t[i]))) ++i;
}

bool parse_string(const std::string &t, size_t &i, std::string &out) {
  skip_ws(t, i);
  if (i >= t.size() || t[i] != '"') return false;
  const size_t e = t.find('"', i + 1);
  if (e == std::string::npos) return false;
  out = t.substr(i + 1, e - i - 1);
  i = e + 1;
  return true;
}

bool expect(const std::string &t, size_t &i, char c) {
  skip_ws(t, i);
  if (i >= t.size() || t[i] != c) return false;
  ++i;
  return true;
}

bool parse_number(const std::string &t, size_t &i, double &v) {
  skip_ws(t, i);
  const char *s = t.c_str() + i;
  char *end = nullptr;
  errno = 0;
  v = std::strtod(s, &end);
  if (end == s || errno != 0) return false;
  i += static_cast<size_t>(end - s);
  return true;
}

// the whole file; false if it cannot be parsed (a missing file is an empty cache)
bool read_cache(const char *path, std::map<std::string, Entry> &out) {
  out.clear();
  FILE *f = std::fopen(path, "rb");
  if (!f) return true;
  std::string t;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) t.append(buf, n);
  std::fclose(f);
  size_t i = 0;
  skip_ws(t, i);
  if (i == t.size()) return true;
  if (!expect(t, i, '{')) return false;
  skip_ws(t, i);
  if (i < t.size() && t[i] == '}') return true;
  for (;;) {
    std::string key;
    if (!parse_string(t, i, key) || !expect(t, i, ':') || !expect(t, i, '{')) return false;
    Entry e;
    skip_ws(t, i);
    if (i < t.size() && t[i] != '}') {
      for (;;) {
        std::string field;
        double v = 0;
        if (!parse_string(t, i, field) || !expect(t, i, ':') || !parse_number(t, i, v)) return false;
        if (field == "cfg") e.cfg = static_cast<int>(v);
        if (field == "box") e.box = static_cast<int>(v);
        if (field == "ms") e.ms = v;
        skip_ws(t, i);
        if (i < t.size() && t[i] == ',') {
          ++i;
          continue;
        }
        break;
      }
    }
    if (!expect(t, i, '}')) return false;
    out[key] = e;
    skip_ws(t, i);
    if (i < t.size() && t[i] == ',') {
      ++i;
      continue;
    }
    return expect(t, i, '}');
  }
}

}  // namespace

namespace tmf {

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string arch = p.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/" + std::to_string(p.multiProcessorCount) + "cu";
}

int tune_cache_lookup(const char *path, const std::string &key, int *cfg, int *box, float *ms) {
  std::map<std::string, Entry> m;
  if (!read_cache(path, m)) return -1;
  auto it = m.find(key);
  if (it == m.end()) return 0;
  *cfg = it->second.cfg;
  *box = it->second.box;
  *ms = static_cast<float>(it->second.ms);
  return 1;
}

tmf_status tune_cache_store(const char *path, const std::string &key, int cfg, int box, float ms) {
  std::map<std::string, Entry> m;
  if (!read_cache(path, m)) return fail(TMF_EINVAL, "tile cache %s is not a cache file this library wrote", path);
  m[key] = Entry{cfg, box, ms};
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return fail(TMF_EINVAL, "cannot write tile cache %s", tmp.c_str());
  std::fprintf(f, "{\n");
  size_t k = 0;
  for (const auto &kv : m) {
    std::fprintf(f, "  \"%s\": {\"cfg\": %d, \"box\": %d, \"ms\": %.6g}%s\n", kv.first.c_str(), kv.second.cfg,
                 kv.second.box, kv.second.ms, ++k < m.size() ? "," : "");
  }
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) return fail(TMF_EINVAL, "cannot write tile cache %s", path);
  return TMF_OK;
}

}  // namespace tmf
