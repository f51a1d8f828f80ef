// The process-wide tuning table (launch choices measured by mtp_solver_tune /
// mtp_batch_tune, keyed by configuration) and its JSON file format:
//   {"format": "mtp-tuning-1",
//    "entries": [{"key": "...", "schedule": 1, "tile_order": 0, "grid_frac": 1.0,
//                 "ms_best": 1.25, "ms_default": 1.5, "candidates": 7}, ...]}
// Unknown members of an entry are ignored; a missing member keeps its default.
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace mtp {

namespace {

std::mutex g_mu;
std::map<std::string, TuneEntry> g_table;

// Minimal JSON reader: objects, arrays, strings, numbers, true/false/null.
struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const std::string& s;
  size_t i = 0;
  explicit JParser(const std::string& src) : s(src) {}
  [[noreturn]] void fail() { throw Error(MTP_ERR_ARG, "tuning file: malformed JSON near byte " + std::to_string(i)); }
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
  void expect(char c) {
    if (!eat(c)) fail();
  }
  std::string string() {
    expect('"');
    std::string out;
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\') {
        if (i >= s.size()) fail();
        const char e = s[i++];
        switch (e) {
          case '"': out += '"'; break;
          case '\\': out += '\\'; break;
          case '/': out += '/'; break;
          case 'n': out += '\n'; break;
          case 't': out += '\t'; break;
          case 'r': out += '\r'; break;
          case 'b': out += '\b'; break;
          case 'f': out += '\f'; break;
          default: fail();   // \u escapes never occur in keys this library writes
        }
      } else {
        out += c;
      }
    }
    if (i >= s.size()) fail();
    ++i;
    return out;
  }
  JVal value(int depth) {
    if (depth > 16) fail();
    ws();
    if (i >= s.size()) fail();
    JVal v;
    const char c = s[i];
    if (c == '{') {
      ++i;
      v.kind = JVal::OBJ;
      if (eat('}')) return v;
      do {
        ws();
        std::string k = string();
        expect(':');
        v.obj.emplace_back(std::move(k), value(depth + 1));
      } while (eat(','));
      expect('}');
    } else if (c == '[') {
      ++i;
      v.kind = JVal::ARR;
      if (eat(']')) return v;
      do {
        v.arr.push_back(value(depth + 1));
      } while (eat(','));
      expect(']');
    } else if (c == '"') {
      v.kind = JVal::STR;
      v.str = string();
    } else if (s.compare(i, 4, "true") == 0) {
      v.kind = JVal::BOOL;
      v.num = 1.0;
      i += 4;
    } else if (s.compare(i, 5, "false") == 0) {
      v.kind = JVal::BOOL;
      i += 5;
    } else if (s.compare(i, 4, "null") == 0) {
      i += 4;
    } else {
      const char* b = s.c_str() + i;
      char* e = nullptr;
      v.kind = JVal::NUM;
      v.num = std::strtod(b, &e);
      if (e == b) fail();
      i += (size_t)(e - b);
    }
    return v;
  }
};

std::string escape(const std::string& k) {
  std::string o;
  for (char c : k) {
    if (c == '"' || c == '\\') o += '\\';
    o += c;
  }
  return o;
}

}  // namespace

bool tune_find(const std::string& key, TuneEntry* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  if (out) *out = it->second;
  return true;
}

void tune_put(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[key] = e;
}

void tune_clear_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
}

int tune_count() {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_table.size();
}

void tune_save_file(const char* path) {
  std::string out = "{\"format\": \"mtp-tuning-1\",\n \"entries\": [";
  {
    std::lock_guard<std::mutex> lk(g_mu);
    bool first = true;
    char buf[512];
    for (const auto& kv : g_table) {
      const TuneEntry& e = kv.second;
      std::snprintf(buf, sizeof(buf),
                    "\"schedule\": %d, \"tile_order\": %d, \"grid_frac\": %.17g, \"ms_best\": %.17g, "
                    "\"ms_default\": %.17g, \"candidates\": %d}",
                    e.schedule, e.tile_order, e.grid_frac, e.ms_best, e.ms_default, e.candidates);
      out += first ? "\n  " : ",\n  ";
      out += "{\"key\": \"" + escape(kv.first) + "\", " + buf;
      first = false;
    }
  }
  out += "\n ]}\n";
  FILE* f = std::fopen(path, "wb");
  if (!f) throw Error(MTP_ERR_ARG, "cannot open the tuning file for writing");
  const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed) throw Error(MTP_ERR_ARG, "tuning file write failed");
}

void tune_load_file(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) throw Error(MTP_ERR_ARG, "cannot open the tuning file");
  std::string src;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) src.append(buf, n);
  std::fclose(f);
  JParser jp(src);
  const JVal root = jp.value(0);
  jp.ws();
  if (jp.i != src.size()) jp.fail();
  const JVal* fmt = root.kind == JVal::OBJ ? root.get("format") : nullptr;
  const JVal* ents = root.kind == JVal::OBJ ? root.get("entries") : nullptr;
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "mtp-tuning-1" || !ents || ents->kind != JVal::ARR)
    throw Error(MTP_ERR_ARG, "tuning file: not an mtp-tuning-1 table");
  std::vector<std::pair<std::string, TuneEntry>> got;
  for (const JVal& e : ents->arr) {
    const JVal* k = e.kind == JVal::OBJ ? e.get("key") : nullptr;
    if (!k || k->kind != JVal::STR) throw Error(MTP_ERR_ARG, "tuning file: entry without a key");
    TuneEntry t;
    auto num = [&](const char* name, double dflt) {
      const JVal* v = e.get(name);
      if (!v) return dflt;
      if (v->kind != JVal::NUM || !std::isfinite(v->num)) throw Error(MTP_ERR_ARG, "tuning file: bad number");
      return v->num;
    };
    t.schedule = (int)num("schedule", 0);
    t.tile_order = (int)num("tile_order", 0);
    t.grid_frac = num("grid_frac", 1.0);
    t.ms_best = num("ms_best", 0.0);
    t.ms_default = num("ms_default", 0.0);
    t.candidates = (int)num("candidates", 0);
    if (t.schedule < 0 || t.schedule > 1 || t.tile_order < 0 || t.tile_order > 3 || !(t.grid_frac > 0.0) ||
        t.grid_frac > 1.0)
      throw Error(MTP_ERR_ARG, "tuning file: choice out of range");
    got.emplace_back(k->str, t);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : got) g_table[kv.first] = kv.second;
}

}  // namespace mtp
