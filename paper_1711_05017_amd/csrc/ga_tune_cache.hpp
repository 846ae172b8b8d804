// ga_tune_cache.hpp -- persisted tuning choices of the correlation path
// (host code only: no HIP types, so that it also builds with a plain C++
// compiler under the host sanitizers).
//
// The cache is a JSON object with one entry per line, keyed by
// "<arch>/<n>/<batch>/<channels>" (e.g. "gfx950/128/64/1"):
//   {
//     "gfx950/128/64/1": {"groups": 4, "k": 4, "xcd": 2, "radix": 0, "overlap": 2, "us": 806.125},
//     ...
//   }
// Readers accept exactly the layout the writer produces; anything else is
// reported as malformed and left untouched.
#pragma once

#include <cctype>
#include <cerrno>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>

#include <unistd.h>

namespace ga {

struct TuneEntry {
  int groups = 4;   // wavefronts of transforms per workgroup in the fused x pass: 4 or 8
  int k = 4;        // batch members per workgroup: 1, 2, 4 or 8
  int xcd = 2;      // 1 XCD-aware grid, 2 plain
  int radix = 0;    // x transforms on the default radix schedule (0) or its alternative (1)
  int overlap = 1;  // parts of the batch over two streams: 1, 2 or 4
  double us = 0.0;  // time per call of this configuration, microseconds
};

inline bool tune_entry_valid(const TuneEntry& e) {
  return (e.groups == 4 || e.groups == 8) && (e.k == 1 || e.k == 2 || e.k == 4 || e.k == 8) &&
         (e.xcd == 1 || e.xcd == 2) && (e.radix == 0 || e.radix == 1) && (e.overlap == 1 || e.overlap == 2 || e.overlap == 4) && e.us >= 0.0 &&
         e.us < 1e12;
}

// "<arch>/<n>/<batch>/<channels>"; the architecture name is cut at its first
// ':' (feature suffixes such as ":sramecc+:xnack-").
inline std::string tune_key(const char* arch, int n, int batch, int channels) {
  std::string a(arch ? arch : "");
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a.resize(colon);
  return a + "/" + std::to_string(n) + "/" + std::to_string(batch) + "/" + std::to_string(channels);
}

inline bool tune_key_valid(const std::string& key) {
  if (key.empty() || key.size() > 200) return false;
  for (char c : key)
    if (!(std::isalnum((unsigned char)c) || c == '/' || c == '_' || c == '-' || c == '.')) return false;
  return true;
}

// Parse the text of a cache; false (and `out` unchanged) if it is not in the
// writer's layout.
inline bool tune_cache_parse(const std::string& text, std::map<std::string, TuneEntry>& out) {
  std::map<std::string, TuneEntry> m;
  size_t pos = 0;
  int state = 0;  // 0 before '{', 1 inside, 2 after '}'
  while (pos < text.size()) {
    size_t eol = text.find('\n', pos);
    if (eol == std::string::npos) eol = text.size();
    std::string line = text.substr(pos, eol - pos);
    pos = eol + 1;
    while (!line.empty() && (line.back() == ' ' || line.back() == '\r' || line.back() == '\t')) line.pop_back();
    size_t lead = 0;
    while (lead < line.size() && (line[lead] == ' ' || line[lead] == '\t')) ++lead;
    line.erase(0, lead);
    if (line.empty()) continue;
    if (state == 0) {
      if (line == "{}") {
        state = 2;
        continue;
      }
      if (line != "{") return false;
      state = 1;
      continue;
    }
    if (state == 2) return false;
    if (line == "}") {
      state = 2;
      continue;
    }
    char key[256] = {0};
    TuneEntry e;
    int used = 0;
    if (std::sscanf(line.c_str(), "\"%255[^\"]\": {\"groups\": %d, \"k\": %d, \"xcd\": %d, \"radix\": %d, \"overlap\": %d, \"us\": %lf}%n",
                    key, &e.groups, &e.k, &e.xcd, &e.radix, &e.overlap, &e.us, &used) != 7)
      return false;
    const std::string rest = line.substr((size_t)used);
    if (!(rest.empty() || rest == ",")) return false;
    if (!tune_key_valid(key) || !tune_entry_valid(e)) return false;
    m[key] = e;
  }
  if (state != 2) return false;
  out.swap(m);
  return true;
}

inline std::string tune_cache_format(const std::map<std::string, TuneEntry>& m) {
  std::string s = "{\n";
  size_t i = 0;
  for (const auto& [key, e] : m) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "  \"%s\": {\"groups\": %d, \"k\": %d, \"xcd\": %d, \"radix\": %d, \"overlap\": %d, \"us\": %.3f}%s\n",
                  key.c_str(), e.groups, e.k, e.xcd, e.radix, e.overlap, e.us, (++i < m.size()) ? "," : "");
    s += buf;
  }
  s += "}\n";
  return s;
}

// Read a cache file. A missing file is an empty cache (exists = false);
// false if the file cannot be read or is malformed.
inline bool tune_cache_load(const char* path, std::map<std::string, TuneEntry>& out, bool& exists) {
  exists = false;
  out.clear();
  FILE* f = std::fopen(path, "rb");
  if (!f) return errno == ENOENT;
  exists = true;
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) {
    text.append(buf, got);
    if (text.size() > (1u << 20)) break;  // a cache is a few KB
  }
  const bool err = std::ferror(f) != 0 || text.size() > (1u << 20);
  std::fclose(f);
  if (err) return false;
  return tune_cache_parse(text, out);
}

// Write the cache: to "<path>.tmp.<pid>" first, then renamed over `path`, so
// that a reader never sees a partly written file.
inline bool tune_cache_store(const char* path, const std::map<std::string, TuneEntry>& m) {
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  const std::string text = tune_cache_format(m);
  const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace ga
