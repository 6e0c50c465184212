// Tile-shape tuning table: reads the JSON file the autotuner writes.
//
//   {"arch": "gfx950", "sweep_pull_kmax": 4096,
//    "entries": [{"class": "sweep", "rhs_max": 256, "group_max": 64, "precision": 0, "shape": 3}, ...]}
//
// Entries are matched in file order (first match wins); "rhs_max",
// "group_max" and "precision" may be omitted (no bound / any precision).
// "sweep_pull_kmax" (optional, integer >= 0) sets the sweeps' pull threshold.
// Other keys are ignored.  A small recursive-descent reader of the JSON subset the file uses (objects,
// arrays, strings without unicode escapes, numbers, true / false / null).
#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <memory>
#include <sstream>

#include "device.h"

namespace hps {

namespace {

struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal *get(const char *k) const {
    for (const auto &kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JReader {
  const std::string &s;
  size_t i = 0;
  int depth = 0;
  explicit JReader(const std::string &t) : s(t) {}
  [[noreturn]] void fail(const char *what) const {
    std::ostringstream o;
    o << "tuning file: " << what << " at byte " << i;
    throw Error{HPS_EINVAL, o.str()};
  }
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  }
  bool lit(const char *w) {
    const size_t n = std::strlen(w);
    if (s.compare(i, n, w) == 0) {
      i += n;
      return true;
    }
    return false;
  }
  std::string str() {
    if (i >= s.size() || s[i] != '"') fail("string expected");
    ++i;
    std::string out;
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\') {
        if (i >= s.size()) fail("bad escape");
        const char e = s[i++];
        c = e == 'n' ? '\n' : e == 't' ? '\t' : e;   // \" \\ \/ and the rest literally
      }
      out.push_back(c);
    }
    if (i >= s.size()) fail("unterminated string");
    ++i;
    return out;
  }
  JVal value() {
    if (++depth > 64) fail("nesting too deep");
    ws();
    JVal v;
    if (i >= s.size()) fail("value expected");
    const char c = s[i];
    if (c == '{') {
      v.kind = JVal::OBJ;
      ++i;
      ws();
      if (i < s.size() && s[i] == '}') {
        ++i;
      } else {
        for (;;) {
          ws();
          std::string k = str();
          ws();
          if (i >= s.size() || s[i] != ':') fail("':' expected");
          ++i;
          v.obj.emplace_back(std::move(k), value());
          ws();
          if (i < s.size() && s[i] == ',') { ++i; continue; }
          if (i < s.size() && s[i] == '}') { ++i; break; }
          fail("',' or '}' expected");
        }
      }
    } else if (c == '[') {
      v.kind = JVal::ARR;
      ++i;
      ws();
      if (i < s.size() && s[i] == ']') {
        ++i;
      } else {
        for (;;) {
          v.arr.push_back(value());
          ws();
          if (i < s.size() && s[i] == ',') { ++i; continue; }
          if (i < s.size() && s[i] == ']') { ++i; break; }
          fail("',' or ']' expected");
        }
      }
    } else if (c == '"') {
      v.kind = JVal::STR;
      v.str = str();
    } else if (lit("true")) {
      v.kind = JVal::BOOL;
      v.num = 1.0;
    } else if (lit("false")) {
      v.kind = JVal::BOOL;
    } else if (lit("null")) {
      v.kind = JVal::NUL;
    } else {
      const char *b = s.c_str() + i;
      char *e = nullptr;
      errno = 0;
      v.num = std::strtod(b, &e);
      if (e == b || errno != 0 || !std::isfinite(v.num)) fail("number expected");
      v.kind = JVal::NUM;
      i += (size_t)(e - b);
    }
    --depth;
    return v;
  }
};

int class_id(const std::string &c) {
  static const char *names[TC_COUNT] = {"sweep", "dinv", "far1", "far2", "near", "schur"};
  for (int k = 0; k < TC_COUNT; ++k)
    if (c == names[k]) return k;
  return -1;
}

}  // namespace

TuneTable read_tuning(const std::string &path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) throw Error{HPS_EIO, "cannot open tuning file " + path};
  std::stringstream buf;
  buf << f.rdbuf();
  const std::string text = buf.str();
  if (text.size() > (1u << 20)) throw Error{HPS_EINVAL, "tuning file larger than 1 MiB: " + path};
  JReader rd(text);
  const JVal root = rd.value();
  rd.ws();
  if (rd.i != text.size()) rd.fail("trailing characters");
  if (root.kind != JVal::OBJ) throw Error{HPS_EINVAL, "tuning file: top level is not an object"};
  const JVal *ent = root.get("entries");
  if (!ent || ent->kind != JVal::ARR) throw Error{HPS_EINVAL, "tuning file: no \"entries\" array"};
  TuneTable table;
  const JVal *pk = root.get("sweep_pull_kmax");
  if (pk && pk->kind != JVal::NUL) {
    if (pk->kind != JVal::NUM || pk->num != std::floor(pk->num) || pk->num < 0 || pk->num > 1.0e15)
      throw Error{HPS_EINVAL, "tuning file: \"sweep_pull_kmax\" must be an integer >= 0"};
    table.sweep_pull_kmax = (int64_t)pk->num;
  }
  std::vector<TuneEntry> &out = table.entries;
  for (const JVal &e : ent->arr) {
    if (e.kind != JVal::OBJ) throw Error{HPS_EINVAL, "tuning file: an entry is not an object"};
    const JVal *c = e.get("class"), *sh = e.get("shape"), *rm = e.get("rhs_max"), *gm = e.get("group_max");
    const JVal *pr = e.get("precision");
    if (!c || c->kind != JVal::STR || class_id(c->str) < 0)
      throw Error{HPS_EINVAL, "tuning file: entry without a known \"class\" (sweep, dinv, far1, far2, near, schur)"};
    if (!sh || sh->kind != JVal::NUM || sh->num != std::floor(sh->num) || sh->num < 0 || sh->num >= TUNE_SHAPES)
      throw Error{HPS_EINVAL, "tuning file: \"shape\" must be an integer 0-12"};
    TuneEntry t;
    t.cls = class_id(c->str);
    t.shape = (int)sh->num;
    t.rhs_max = std::numeric_limits<int64_t>::max();
    t.group_max = std::numeric_limits<double>::infinity();
    if (rm && rm->kind != JVal::NUL) {
      if (rm->kind != JVal::NUM || rm->num < 0) throw Error{HPS_EINVAL, "tuning file: bad \"rhs_max\""};
      if (rm->num < 9.0e18) t.rhs_max = (int64_t)rm->num;
    }
    if (gm && gm->kind != JVal::NUL) {
      if (gm->kind != JVal::NUM || gm->num < 0) throw Error{HPS_EINVAL, "tuning file: bad \"group_max\""};
      t.group_max = gm->num;
    }
    if (pr && pr->kind != JVal::NUL) {
      if (pr->kind != JVal::NUM || pr->num != std::floor(pr->num) || pr->num < 0 || pr->num > 2)
        throw Error{HPS_EINVAL, "tuning file: \"precision\" must be 0, 1 or 2"};
      t.precision = (int)pr->num;
    }
    out.push_back(t);
  }
  return table;
}

}  // namespace hps
