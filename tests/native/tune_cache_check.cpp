// Host checks of the tuning cache (paper_1711_05017_amd/csrc/ga_tune_cache.hpp),
// built with the host sanitizers by tests/test_tune_cache.py. Prints one line
// per check and exits non-zero on the first failure. argv[1]: a scratch
// directory.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "ga_tune_cache.hpp"

using namespace ga;

static int fails = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                   \
    }                                                            \
  } while (0)

static std::string slurp(const std::string& path) {
  std::string s;
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return s;
  char buf[1024];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, got);
  std::fclose(f);
  return s;
}

static void spit(const std::string& path, const std::string& text) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) return;
  std::fwrite(text.data(), 1, text.size(), f);
  std::fclose(f);
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const std::string dir = argv[1];
  // keys
  CHECK(tune_key("gfx950:sramecc+:xnack-", 128, 64, 1) == "gfx950/128/64/1");
  CHECK(tune_key("gfx950", 96, 3, 1) == "gfx950/96/3/1");
  CHECK(tune_key(nullptr, 16, 1, 1) == "/16/1/1");
  CHECK(!tune_key_valid("") && !tune_key_valid("a\"b") && tune_key_valid("gfx950/128/64/1"));
  // round trip, sorted keys, the empty cache
  std::map<std::string, TuneEntry> m, back;
  CHECK(tune_cache_parse("{}\n", back) && back.empty());
  CHECK(tune_cache_parse(tune_cache_format(m), back) && back.empty());
  m["gfx950/128/64/1"] = TuneEntry{4, 4, 2, 0, 2, 806.125};
  m["gfx950/64/16/1"] = TuneEntry{8, 1, 1, 1, 1, 40.5};
  const std::string text = tune_cache_format(m);
  CHECK(tune_cache_parse(text, back) && back.size() == 2);
  CHECK(back["gfx950/128/64/1"].groups == 4 && back["gfx950/128/64/1"].overlap == 2 &&
        back["gfx950/128/64/1"].us == 806.125 && back["gfx950/128/64/1"].radix == 0);
  CHECK(back["gfx950/64/16/1"].groups == 8 && back["gfx950/64/16/1"].k == 1 && back["gfx950/64/16/1"].xcd == 1 &&
        back["gfx950/64/16/1"].radix == 1);
  // malformed text: refused, the output left as it was
  const char* bad[] = {
      "",
      "{",
      "[]\n",
      "{\n}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": 1.0}\n",  // no closing brace
      "{\n  \"k\": {\"groups\": 5, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": 1.0}\n}\n",  // groups out of range
      "{\n  \"k\": {\"groups\": 4, \"k\": 3, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": 1.0}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 0, \"radix\": 0, \"overlap\": 2, \"us\": 1.0}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 3, \"us\": 1.0}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": nan}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": -1}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": 1.0} junk\n}\n",
      "{\n  \"a b\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": 1.0}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 2, \"overlap\": 2, \"us\": 1.0}\n}\n",
      "{\n  \"k\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"overlap\": 2, \"us\": 1.0}\n}\n",  // no radix
      "{\"gfx950/64/4/1\": {\"groups\": 4}}\n",
  };
  for (const char* b : bad) {
    std::map<std::string, TuneEntry> keep = back;
    CHECK(!tune_cache_parse(b, keep));
    CHECK(keep.size() == back.size());
  }
  // a key longer than the parser's buffer is refused, not truncated
  CHECK(!tune_cache_parse("{\n  \"" + std::string(300, 'a') +
                              "\": {\"groups\": 4, \"k\": 4, \"xcd\": 2, \"radix\": 0, \"overlap\": 2, \"us\": 1.0}\n}\n",
                          back));
  // files: a missing file is an empty cache; store then load; merge of a new key
  const std::string path = dir + "/tune.json";
  bool exists = true;
  std::map<std::string, TuneEntry> loaded;
  CHECK(tune_cache_load(path.c_str(), loaded, exists) && !exists && loaded.empty());
  CHECK(tune_cache_store(path.c_str(), m));
  CHECK(tune_cache_load(path.c_str(), loaded, exists) && exists && loaded.size() == 2);
  loaded["gfx950/192/8/1"] = TuneEntry{4, 2, 2, 0, 4, 1234.5};
  CHECK(tune_cache_store(path.c_str(), loaded));
  CHECK(tune_cache_load(path.c_str(), back, exists) && back.size() == 3 && back["gfx950/192/8/1"].overlap == 4);
  // a malformed file is reported and not rewritten by the caller
  const std::string badpath = dir + "/bad.json";
  spit(badpath, "not json\n");
  CHECK(!tune_cache_load(badpath.c_str(), back, exists) && exists);
  CHECK(slurp(badpath) == "not json\n");
  // a directory that does not exist: store fails and leaves no file
  CHECK(!tune_cache_store((dir + "/missing/tune.json").c_str(), m));
  std::printf("%s\n", fails ? "FAILED" : "OK");
  std::fputs(slurp(path).c_str(), stdout);
  return fails ? 1 : 0;
}
