// Host-side cache of autotuned schedules: the schedule name a plan's
// autotuner chose, keyed by the device and the plan's shape, kept in a small
// JSON file so that a later plan of the same shape (in this process or
// another) starts on it without timing again.
//
// File format (version 1), written whole on every store:
//
//   {"qft_schedule_cache": 1, "entries": {
//     "<key>": "<schedule name>",
//     ...
//   }}
//
// Keys and names never contain '"' or '\\' (they are built from device
// names, sizes and the library's schedule names).  A file that does not
// parse, has another version, or names a schedule the plan does not have is
// ignored: deleting or corrupting the file only costs a re-tune.
//
// Location: $QFT_SCHEDULE_CACHE if set ("off" or empty disables the cache),
// else $XDG_CACHE_HOME/qft-gfx950/schedules.json, else
// $HOME/.cache/qft-gfx950/schedules.json.
#pragma once

#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

namespace qftk {

constexpr int kScheduleCacheVersion = 1;

inline std::string schedule_cache_path() {
  if (const char* p = std::getenv("QFT_SCHEDULE_CACHE")) {
    const std::string s(p);
    if (s.empty() || s == "off") return std::string();
    return s;
  }
  std::string dir;
  if (const char* x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
  else if (const char* h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
  else return std::string();
  return dir + "/qft-gfx950/schedules.json";
}

// Parses the file; false if it is missing, malformed or of another version.
inline bool schedule_cache_read(const std::string& path,
                                std::map<std::string, std::string>& out) {
  out.clear();
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0 && txt.size() < (1u << 24)) txt.append(buf, n);
  std::fclose(f);
  // version
  const std::string vtag = "\"qft_schedule_cache\":";
  size_t p = txt.find(vtag);
  if (p == std::string::npos) return false;
  p += vtag.size();
  while (p < txt.size() && txt[p] == ' ') ++p;
  if (std::atoi(txt.c_str() + p) != kScheduleCacheVersion) return false;
  p = txt.find("\"entries\"", p);
  if (p == std::string::npos) return false;
  p = txt.find('{', p);
  if (p == std::string::npos) return false;
  // "key": "value" pairs until the closing brace
  auto str = [&](size_t& i, std::string& s) {
    while (i < txt.size() && (txt[i] == ' ' || txt[i] == '\n' || txt[i] == '\r' ||
                              txt[i] == '\t' || txt[i] == ','))
      ++i;
    if (i >= txt.size() || txt[i] != '"') return false;
    const size_t e = txt.find('"', i + 1);
    if (e == std::string::npos) return false;
    s = txt.substr(i + 1, e - i - 1);
    i = e + 1;
    return true;
  };
  size_t i = p + 1;
  for (;;) {
    size_t j = i;
    while (j < txt.size() && (txt[j] == ' ' || txt[j] == '\n' || txt[j] == '\r' ||
                              txt[j] == '\t' || txt[j] == ','))
      ++j;
    if (j < txt.size() && txt[j] == '}') return true;
    std::string k, v;
    if (!str(i, k)) return false;
    while (i < txt.size() && txt[i] == ' ') ++i;
    if (i >= txt.size() || txt[i] != ':') return false;
    ++i;
    while (i < txt.size() && txt[i] == ' ') ++i;
    if (!str(i, v)) return false;
    out[k] = v;
  }
}

inline bool schedule_cache_lookup(const std::string& path, const std::string& key,
                                  std::string& name) {
  std::map<std::string, std::string> m;
  if (!schedule_cache_read(path, m)) return false;
  const auto it = m.find(key);
  if (it == m.end()) return false;
  name = it->second;
  return true;
}

inline bool cache_text_ok(const std::string& s) {
  return s.find('"') == std::string::npos && s.find('\\') == std::string::npos &&
         s.find('\n') == std::string::npos;
}

// Merges key -> name into the file (creating its directory); a file that
// does not parse is replaced.  Writes a temporary file and renames it over
// the old one.  Returns false if the cache is disabled or the write fails.
inline bool schedule_cache_store(const std::string& path, const std::string& key,
                                 const std::string& name) {
  if (path.empty() || !cache_text_ok(key) || !cache_text_ok(name)) return false;
  std::map<std::string, std::string> m;
  schedule_cache_read(path, m);
  m[key] = name;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0) {
    // mkdir -p of the directory
    std::string dir = path.substr(0, slash);
    for (size_t q = 1; q <= dir.size(); ++q) {
      if (q == dir.size() || dir[q] == '/') {
        const std::string part = dir.substr(0, q);
        if (::mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return false;
      }
    }
  }
  const std::string tmp = path + ".tmp" + std::to_string((long)::getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{\"qft_schedule_cache\": %d, \"entries\": {", kScheduleCacheVersion);
  bool first = true;
  for (const auto& kv : m) {
    std::fprintf(f, "%s\n  \"%s\": \"%s\"", first ? "" : ",", kv.first.c_str(),
                 kv.second.c_str());
    first = false;
  }
  std::fprintf(f, "\n}}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace qftk
