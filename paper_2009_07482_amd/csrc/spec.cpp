// The specification-file frontend (Sec. IV-A): a dag.json text lowered onto the DAG calls of the
// C ABI.  The file lists kernels (id, name, dev, buffer tuples <type, size, pos> in
// inputBuffers / outputBuffers, variable-argument tuples <type, pos, value>, globalWorkSize),
// the task-component partition tc, the command-queue counts cq and the edges
// "k_i,b_r -> k_j,b_s" whose buffer ids are argument positions.  Sizes, work sizes and argument
// values may be symbolic expressions over symbols bound when the file is loaded.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "core.hpp"

namespace psc {
namespace {

// ---- a small JSON reader (RFC 8259 values; numbers kept as double and as their text) ----------
struct Json {
  enum Type { Null, Bool, Num, Str, Arr, Obj } type = Null;
  bool b = false;
  double num = 0;
  std::string str;                                     // Str, and a number's text
  std::vector<Json> arr;
  std::vector<std::pair<std::string, Json>> obj;       // in file order

  const Json *get(const std::string &k) const {
    for (const auto &kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

class Reader {
 public:
  explicit Reader(const char *t) : s_(t) {}
  Json document() {
    Json v = value(0);
    ws();
    if (s_[i_]) err("text after the JSON value");
    return v;
  }

 private:
  const char *s_;
  size_t i_ = 0;

  [[noreturn]] void err(const std::string &m) const {
    size_t line = 1, col = 1;
    for (size_t k = 0; k < i_ && s_[k]; ++k) {
      if (s_[k] == '\n') ++line, col = 1;
      else ++col;
    }
    fail(PSC_ERR_ARG, "dag spec: JSON " + m + " at line " + std::to_string(line) + ", column " + std::to_string(col));
  }
  void ws() {
    while (s_[i_] == ' ' || s_[i_] == '\t' || s_[i_] == '\n' || s_[i_] == '\r') ++i_;
  }
  bool lit(const char *w) {
    const size_t n = std::strlen(w);
    if (std::strncmp(s_ + i_, w, n) != 0) return false;
    i_ += n;
    return true;
  }
  Json value(int depth) {
    if (depth > 64) err("nesting too deep");
    ws();
    Json v;
    const char c = s_[i_];
    if (c == '{') {
      v.type = Json::Obj;
      ++i_;
      ws();
      if (s_[i_] == '}') { ++i_; return v; }
      for (;;) {
        ws();
        if (s_[i_] != '"') err("expects a string key");
        std::string k = string();
        ws();
        if (s_[i_] != ':') err("expects ':'");
        ++i_;
        v.obj.emplace_back(std::move(k), value(depth + 1));
        ws();
        if (s_[i_] == ',') { ++i_; continue; }
        if (s_[i_] == '}') { ++i_; return v; }
        err("expects ',' or '}'");
      }
    }
    if (c == '[') {
      v.type = Json::Arr;
      ++i_;
      ws();
      if (s_[i_] == ']') { ++i_; return v; }
      for (;;) {
        v.arr.push_back(value(depth + 1));
        ws();
        if (s_[i_] == ',') { ++i_; continue; }
        if (s_[i_] == ']') { ++i_; return v; }
        err("expects ',' or ']'");
      }
    }
    if (c == '"') {
      v.type = Json::Str;
      v.str = string();
      return v;
    }
    if (lit("true")) { v.type = Json::Bool; v.b = true; return v; }
    if (lit("false")) { v.type = Json::Bool; return v; }
    if (lit("null")) return v;
    if (c == '-' || std::isdigit(static_cast<unsigned char>(c))) {
      const size_t a = i_;
      if (s_[i_] == '-') ++i_;
      if (!std::isdigit(static_cast<unsigned char>(s_[i_]))) err("malformed number");
      while (std::isdigit(static_cast<unsigned char>(s_[i_]))) ++i_;
      if (s_[i_] == '.') {
        ++i_;
        if (!std::isdigit(static_cast<unsigned char>(s_[i_]))) err("malformed number");
        while (std::isdigit(static_cast<unsigned char>(s_[i_]))) ++i_;
      }
      if (s_[i_] == 'e' || s_[i_] == 'E') {
        ++i_;
        if (s_[i_] == '+' || s_[i_] == '-') ++i_;
        if (!std::isdigit(static_cast<unsigned char>(s_[i_]))) err("malformed number");
        while (std::isdigit(static_cast<unsigned char>(s_[i_]))) ++i_;
      }
      v.type = Json::Num;
      v.str.assign(s_ + a, i_ - a);
      v.num = std::strtod(v.str.c_str(), nullptr);
      return v;
    }
    err("unexpected character");
  }
  std::string string() {
    ++i_;  // opening quote
    std::string out;
    for (;;) {
      const unsigned char c = static_cast<unsigned char>(s_[i_]);
      if (!c) err("unterminated string");
      if (c < 0x20) err("control character in a string");
      ++i_;
      if (c == '"') return out;
      if (c != '\\') { out.push_back(char(c)); continue; }
      const char e = s_[i_++];
      switch (e) {
        case '"': out.push_back('"'); break;
        case '\\': out.push_back('\\'); break;
        case '/': out.push_back('/'); break;
        case 'b': out.push_back('\b'); break;
        case 'f': out.push_back('\f'); break;
        case 'n': out.push_back('\n'); break;
        case 'r': out.push_back('\r'); break;
        case 't': out.push_back('\t'); break;
        case 'u': {
          unsigned cp = 0;
          for (int k = 0; k < 4; ++k) {
            const char h = s_[i_++];
            cp <<= 4;
            if (h >= '0' && h <= '9') cp |= unsigned(h - '0');
            else if (h >= 'a' && h <= 'f') cp |= unsigned(h - 'a' + 10);
            else if (h >= 'A' && h <= 'F') cp |= unsigned(h - 'A' + 10);
            else err("bad \\u escape");
          }
          if (cp < 0x80) {
            out.push_back(char(cp));
          } else if (cp < 0x800) {
            out.push_back(char(0xC0 | (cp >> 6)));
            out.push_back(char(0x80 | (cp & 0x3F)));
          } else {
            out.push_back(char(0xE0 | (cp >> 12)));
            out.push_back(char(0x80 | ((cp >> 6) & 0x3F)));
            out.push_back(char(0x80 | (cp & 0x3F)));
          }
          break;
        }
        default: err("bad escape");
      }
    }
  }
};

// ---- symbolic expressions: + - * / % and parentheses over numbers and bound symbols ----------
class Expr {
 public:
  Expr(const std::string &text, const std::map<std::string, double> &sym, const std::string &where)
      : t_(text), sym_(sym), where_(where) {}
  double eval() {
    const double v = sum();
    ws();
    if (i_ != t_.size()) err("unexpected '" + t_.substr(i_) + "'");
    return v;
  }

 private:
  const std::string &t_;
  const std::map<std::string, double> &sym_;
  const std::string &where_;
  size_t i_ = 0;

  [[noreturn]] void err(const std::string &m) const {
    fail(PSC_ERR_ARG, "dag spec: " + where_ + ": expression \"" + t_ + "\": " + m);
  }
  void ws() {
    while (i_ < t_.size() && std::isspace(static_cast<unsigned char>(t_[i_]))) ++i_;
  }
  double sum() {
    double v = product();
    for (;;) {
      ws();
      if (i_ < t_.size() && (t_[i_] == '+' || t_[i_] == '-')) {
        const char op = t_[i_++];
        const double r = product();
        v = op == '+' ? v + r : v - r;
      } else {
        return v;
      }
    }
  }
  double product() {
    double v = unary();
    for (;;) {
      ws();
      if (i_ < t_.size() && (t_[i_] == '*' || t_[i_] == '/' || t_[i_] == '%')) {
        const char op = t_[i_++];
        const double r = unary();
        if (op == '*') {
          v *= r;
        } else {
          if (r == 0) err("division by zero");
          v = op == '/' ? v / r : std::fmod(v, r);
        }
      } else {
        return v;
      }
    }
  }
  double unary() {
    ws();
    if (i_ < t_.size() && t_[i_] == '-') { ++i_; return -unary(); }
    if (i_ < t_.size() && t_[i_] == '+') { ++i_; return unary(); }
    if (i_ < t_.size() && t_[i_] == '(') {
      ++i_;
      const double v = sum();
      ws();
      if (i_ >= t_.size() || t_[i_] != ')') err("missing ')'");
      ++i_;
      return v;
    }
    if (i_ < t_.size() && (std::isdigit(static_cast<unsigned char>(t_[i_])) || t_[i_] == '.')) {
      char *end = nullptr;
      const double v = std::strtod(t_.c_str() + i_, &end);
      i_ = size_t(end - t_.c_str());
      return v;
    }
    if (i_ < t_.size() && (std::isalpha(static_cast<unsigned char>(t_[i_])) || t_[i_] == '_')) {
      const size_t a = i_;
      while (i_ < t_.size() && (std::isalnum(static_cast<unsigned char>(t_[i_])) || t_[i_] == '_')) ++i_;
      const std::string name = t_.substr(a, i_ - a);
      auto it = sym_.find(name);
      if (it == sym_.end()) err("unbound symbol '" + name + "'");
      return it->second;
    }
    err(i_ < t_.size() ? "unexpected '" + t_.substr(i_) + "'" : "ends early");
  }
};

double number(const Json &v, const std::map<std::string, double> &sym, const std::string &where) {
  if (v.type == Json::Num) return v.num;
  if (v.type == Json::Str) return Expr(v.str, sym, where).eval();
  fail(PSC_ERR_ARG, "dag spec: " + where + ": expects a number or an expression");
}

int64_t integer(const Json &v, const std::map<std::string, double> &sym, const std::string &where) {
  const double x = number(v, sym, where);
  if (!(std::fabs(x) < 9.0e15) || x != std::floor(x))
    fail(PSC_ERR_ARG, "dag spec: " + where + ": " + std::to_string(x) + " is not an integer");
  return int64_t(x);
}

const Json &member(const Json &o, const char *k, const std::string &where) {
  const Json *v = o.type == Json::Obj ? o.get(k) : nullptr;
  if (!v) fail(PSC_ERR_ARG, "dag spec: " + where + " has no \"" + k + "\"");
  return *v;
}

int32_t dtype_of(const std::string &t, const std::string &where) {
  if (t == "float" || t == "f32" || t == "float32") return PSC_F32;
  if (t == "bfloat16" || t == "bf16") return PSC_BF16;
  fail(PSC_ERR_ARG, "dag spec: " + where + ": element type \"" + t + "\" (float or bfloat16)");
}

// Kernel names of the spec and the library kind each one runs.
int32_t kind_of(const std::string &name, const std::string &where) {
  if (name == "gemm" || name == "matmul") return PSC_GEMM;
  if (name == "transpose") return PSC_TRANSPOSE;
  if (name == "softmax") return PSC_SOFTMAX;
  if (name == "add" || name == "vadd") return PSC_ADD;
  fail(PSC_ERR_UNSUPPORTED, "dag spec: " + where + ": no kernel named \"" + name +
                                "\" (gemm/matmul, transpose, softmax, add/vadd)");
}

struct Arg {           // one buffer argument of one kernel
  int32_t kernel = 0, pos = 0;
  bool output = false;
  int32_t dtype = PSC_F32;
  int64_t rows = 0, cols = 0;
  std::string name;    // "name" field, or empty
  std::string view_of;
  int64_t row_off = 0, col_off = 0;
};

struct Root {          // a top-level "buffers" entry: storage that arguments may window
  std::string name;
  int32_t dtype = PSC_F32;
  int64_t rows = 0, cols = 0;
};

int32_t find_root(std::vector<int32_t> &up, int32_t x) {
  while (up[x] != x) x = up[x] = up[up[x]];
  return x;
}

}  // namespace
}  // namespace psc

namespace psc {

// Parses and lowers a specification file (see psc_dag_from_json in psc.h); throws psc::Error,
// leaving nothing allocated.
psc_dag *dag_from_json(const char *json, const char *const *sym_names, const int64_t *sym_values, int32_t n_sym,
                       psc_spec_info *info) {
  psc_dag *dag = nullptr;
  // the ABI calls below report through the library's thread-local message
  auto abi = [&](psc_status st) {
    if (st != PSC_OK) fail(st, psc_last_error());
  };
  try {
    if (!json) fail(PSC_ERR_ARG, "NULL argument");
    if (n_sym < 0 || (n_sym > 0 && (!sym_names || !sym_values))) fail(PSC_ERR_ARG, "bad symbol list");
    const Json doc = Reader(json).document();
    if (doc.type != Json::Obj) fail(PSC_ERR_ARG, "dag spec: the document is not an object");
    // symbols: the file's defaults, then the caller's values (the run-time binding of Sec. IV-A)
    std::map<std::string, double> sym;
    if (const Json *s = doc.get("symbols")) {
      if (s->type != Json::Obj) fail(PSC_ERR_ARG, "dag spec: \"symbols\" is not an object");
      for (const auto &kv : s->obj) sym[kv.first] = number(kv.second, sym, "symbol " + kv.first);
    }
    for (int32_t i = 0; i < n_sym; ++i) {
      if (!sym_names[i] || !*sym_names[i]) fail(PSC_ERR_ARG, "empty symbol name");
      sym[sym_names[i]] = double(sym_values[i]);
    }
    // top-level storage that kernel arguments may window
    std::vector<Root> roots;
    std::map<std::string, int32_t> root_by_name;
    if (const Json *bl = doc.get("buffers")) {
      if (bl->type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: \"buffers\" is not a list");
      for (const Json &b : bl->arr) {
        Root r;
        const std::string where = "buffers entry " + std::to_string(roots.size());
        const Json &nm = member(b, "name", where);
        if (nm.type != Json::Str || nm.str.empty()) fail(PSC_ERR_ARG, "dag spec: " + where + ": bad name");
        r.name = nm.str;
        r.dtype = dtype_of(member(b, "type", where).str, where);
        r.rows = integer(member(b, "rows", where), sym, where + " rows");
        r.cols = integer(member(b, "cols", where), sym, where + " cols");
        if (root_by_name.count(r.name)) fail(PSC_ERR_NAME, "dag spec: duplicate buffer \"" + r.name + "\"");
        root_by_name[r.name] = int32_t(roots.size());
        roots.push_back(r);
      }
    }
    const Json &kl = member(doc, "kernels", "the document");
    if (kl.type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: \"kernels\" is not a list");
    const int32_t nk = int32_t(kl.arr.size());
    // kernels in id order; ids must be 0..n-1
    std::vector<const Json *> by_id(nk, nullptr);
    for (const Json &k : kl.arr) {
      const int64_t id = integer(member(k, "id", "a kernel"), sym, "kernel id");
      if (id < 0 || id >= nk || by_id[id]) fail(PSC_ERR_ARG, "dag spec: kernel ids must be 0..n-1, each once");
      by_id[id] = &k;
    }
    std::vector<int32_t> kind(nk);
    std::vector<float> alpha(nk, 1.0f);
    std::vector<std::string> kname(nk);
    std::vector<Arg> args;
    std::vector<std::map<int32_t, int32_t>> arg_at(nk);   // kernel -> pos -> index in args
    for (int32_t k = 0; k < nk; ++k) {
      const Json &K = *by_id[k];
      const std::string where = "kernel " + std::to_string(k);
      const Json &nm = member(K, "name", where);
      if (nm.type != Json::Str) fail(PSC_ERR_ARG, "dag spec: " + where + ": name is not a string");
      kind[k] = kind_of(nm.str, where);
      if (const Json *dev = K.get("dev"))
        if (!(dev->type == Json::Str && dev->str == "gpu"))
          fail(PSC_ERR_UNSUPPORTED, "dag spec: " + where + " asks for device \"" + dev->str +
                                        "\"; this executor maps every kernel to the one GPU");
      if (const Json *io = K.get("ioBuffers"))
        if (!(io->type == Json::Arr && io->arr.empty()))
          fail(PSC_ERR_UNSUPPORTED, "dag spec: " + where + ": ioBuffers (a buffer both read and written) "
                                    "is not a kind of argument the library's kernels take");
      // variable arguments in position order give the dimensions: gemm M, N, K [, alpha];
      // transpose, softmax and add R, C
      std::vector<std::pair<int64_t, const Json *>> vars;
      if (const Json *va = K.get("varArguments")) {
        if (va->type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: " + where + ": varArguments is not a list");
        for (const Json &v : va->arr)
          vars.push_back({integer(member(v, "pos", where + " variable argument"), sym, where + " pos"), &v});
      }
      std::sort(vars.begin(), vars.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
      std::vector<int64_t> dims;
      for (const auto &pv : vars) {
        const Json &v = *pv.second;
        const std::string vt = v.get("type") && v.get("type")->type == Json::Str ? v.get("type")->str : "int";
        const std::string w = where + " variable argument at pos " + std::to_string(pv.first);
        if (vt == "float" || vt == "double") {
          if (kind[k] != PSC_GEMM) fail(PSC_ERR_ARG, "dag spec: " + w + ": only gemm takes a float (alpha)");
          alpha[k] = float(number(member(v, "value", w), sym, w));
        } else {
          dims.push_back(integer(member(v, "value", w), sym, w));
        }
      }
      const size_t want = kind[k] == PSC_GEMM ? 3 : 2;
      if (dims.size() != want)
        fail(PSC_ERR_ARG, "dag spec: " + where + ": " + nm.str + " takes " + std::to_string(want) +
                              " integer variable arguments (" + (want == 3 ? "M, N, K" : "rows, cols") + "), got " +
                              std::to_string(dims.size()));
      for (int64_t x : dims)
        if (x < 0 || x >= (int64_t(1) << 31)) fail(PSC_ERR_ARG, "dag spec: " + where + ": dimension out of range");
      // the work size is the kernel's own business here (each kernel picks its grid), but its
      // expressions must evaluate; "src" (the kernel's source file) names nothing to load
      if (const Json *wd = K.get("workDimension")) {
        const int64_t d = integer(*wd, sym, where + " workDimension");
        if (d < 1 || d > 3) fail(PSC_ERR_ARG, "dag spec: " + where + ": workDimension must be 1, 2 or 3");
      }
      if (const Json *gw = K.get("globalWorkSize")) {
        if (gw->type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: " + where + ": globalWorkSize is not a list");
        for (const Json &x : gw->arr) (void)integer(x, sym, where + " globalWorkSize");
      }
      // buffer arguments in position order: inputs then the output, with the kind's shapes
      std::vector<std::pair<int64_t, std::pair<const Json *, bool>>> bufs;
      for (const char *key : {"inputBuffers", "outputBuffers"}) {
        const Json &bl2 = member(K, key, where);
        if (bl2.type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: " + where + ": " + key + " is not a list");
        for (const Json &b : bl2.arr)
          bufs.push_back({integer(member(b, "pos", where + " buffer"), sym, where + " buffer pos"),
                          {&b, std::strcmp(key, "outputBuffers") == 0}});
      }
      std::sort(bufs.begin(), bufs.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
      const int n_in = (kind[k] == PSC_GEMM || kind[k] == PSC_ADD) ? 2 : 1;
      int seen_in = 0, seen_out = 0;
      for (const auto &pb : bufs) (pb.second.second ? seen_out : seen_in)++;
      if (seen_in != n_in || seen_out != 1)
        fail(PSC_ERR_ARG, "dag spec: " + where + ": " + nm.str + " takes " + std::to_string(n_in) +
                              " input buffer(s) and 1 output buffer");
      std::vector<std::pair<int64_t, int64_t>> shapes;   // in position order: inputs, then output
      if (kind[k] == PSC_GEMM) shapes = {{dims[0], dims[2]}, {dims[2], dims[1]}, {dims[0], dims[1]}};
      else if (kind[k] == PSC_TRANSPOSE) shapes = {{dims[0], dims[1]}, {dims[1], dims[0]}};
      else if (kind[k] == PSC_SOFTMAX) shapes = {{dims[0], dims[1]}, {dims[0], dims[1]}};
      else shapes = {{dims[0], dims[1]}, {dims[0], dims[1]}, {dims[0], dims[1]}};
      for (size_t j = 0; j < bufs.size(); ++j) {
        const Json &b = *bufs[j].second.first;
        Arg a;
        a.kernel = k;
        a.pos = int32_t(bufs[j].first);
        a.output = bufs[j].second.second;
        if (a.output != (j + 1 == bufs.size()))
          fail(PSC_ERR_ARG, "dag spec: " + where + ": the output buffer must follow the inputs in position order");
        const std::string w = where + " buffer at pos " + std::to_string(a.pos);
        if (arg_at[k].count(a.pos)) fail(PSC_ERR_ARG, "dag spec: " + w + " is listed twice");
        const Json &ty = member(b, "type", w);
        a.dtype = dtype_of(ty.type == Json::Str ? ty.str : "", w);
        a.rows = shapes[j].first;
        a.cols = shapes[j].second;
        const int64_t size = integer(member(b, "size", w), sym, w + " size");
        if (size != a.rows * a.cols)
          fail(PSC_ERR_SHAPE, "dag spec: " + w + ": size " + std::to_string(size) + " but " + nm.str + " with these "
                              "arguments needs " + std::to_string(a.rows) + " x " + std::to_string(a.cols));
        if (const Json *n2 = b.get("name")) a.name = n2->str;
        if (const Json *vo = b.get("view_of")) {
          a.view_of = vo->str;
          if (!root_by_name.count(a.view_of))
            fail(PSC_ERR_NAME, "dag spec: " + w + ": view_of names no entry of \"buffers\"");
          if (const Json *x = b.get("row_off")) a.row_off = integer(*x, sym, w + " row_off");
          if (const Json *x = b.get("col_off")) a.col_off = integer(*x, sym, w + " col_off");
        }
        if (!a.name.empty() && root_by_name.count(a.name) && !a.view_of.empty())
          fail(PSC_ERR_NAME, "dag spec: " + w + ": a view cannot take the name of a buffers entry");
        arg_at[k][a.pos] = int32_t(args.size());
        args.push_back(a);
      }
      kname[k] = nm.str + "_" + std::to_string(k);
    }
    // edges k_i,b_r -> k_j,b_s (argument positions)
    struct Edge { int32_t ki, br, kj, bs; };
    std::vector<Edge> edges;
    if (const Json *el = doc.get("edges")) {
      if (el->type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: \"edges\" is not a list");
      for (const Json &e : el->arr) {
        Edge x{};
        if (e.type == Json::Str) {
          int a0, a1, a2, a3;
          char tail = 0;
          if (std::sscanf(e.str.c_str(), " %d , %d -> %d , %d %c", &a0, &a1, &a2, &a3, &tail) != 4)
            fail(PSC_ERR_ARG, "dag spec: edge \"" + e.str + "\" is not of the form \"k_i,b_r -> k_j,b_s\"");
          x = {a0, a1, a2, a3};
        } else if (e.type == Json::Arr && e.arr.size() == 4) {
          x = {int32_t(integer(e.arr[0], sym, "edge")), int32_t(integer(e.arr[1], sym, "edge")),
               int32_t(integer(e.arr[2], sym, "edge")), int32_t(integer(e.arr[3], sym, "edge"))};
        } else {
          fail(PSC_ERR_ARG, "dag spec: an edge is a string \"k_i,b_r -> k_j,b_s\" or a list of four integers");
        }
        const std::string w = "edge " + std::to_string(x.ki) + "," + std::to_string(x.br) + " -> " +
                              std::to_string(x.kj) + "," + std::to_string(x.bs);
        if (x.ki < 0 || x.ki >= nk || x.kj < 0 || x.kj >= nk) fail(PSC_ERR_ARG, "dag spec: " + w + ": no such kernel");
        if (!arg_at[x.ki].count(x.br) || !args[arg_at[x.ki][x.br]].output)
          fail(PSC_ERR_NAME, "dag spec: " + w + ": argument " + std::to_string(x.br) + " is not an output of kernel " +
                                 std::to_string(x.ki));
        if (!arg_at[x.kj].count(x.bs) || args[arg_at[x.kj][x.bs]].output)
          fail(PSC_ERR_NAME, "dag spec: " + w + ": argument " + std::to_string(x.bs) + " is not an input of kernel " +
                                 std::to_string(x.kj));
        edges.push_back(x);
      }
    }
    // one device buffer per class of arguments joined by edges or by a shared name
    const int32_t na = int32_t(args.size());
    std::vector<int32_t> up(na);
    std::iota(up.begin(), up.end(), 0);
    std::map<std::string, int32_t> first_named;
    for (int32_t i = 0; i < na; ++i) {
      if (args[i].name.empty()) continue;
      auto it = first_named.find(args[i].name);
      if (it == first_named.end()) first_named[args[i].name] = i;
      else up[find_root(up, i)] = find_root(up, it->second);
    }
    for (const Edge &e : edges) up[find_root(up, arg_at[e.ki][e.br])] = find_root(up, arg_at[e.kj][e.bs]);
    std::map<int32_t, std::vector<int32_t>> cls;
    for (int32_t i = 0; i < na; ++i) cls[find_root(up, i)].push_back(i);
    std::vector<std::string> arg_buf(na);
    std::set<std::string> used_names;
    for (const Root &r : roots) used_names.insert(r.name);
    struct NewBuf { std::string name; const Arg *a; };
    std::vector<NewBuf> to_add;
    for (auto &c : cls) {
      const std::vector<int32_t> &m = c.second;
      std::string nm;
      const Arg *rep = &args[m[0]];
      for (int32_t i : m) {
        const Arg &a = args[i];
        if (!a.name.empty() && nm.empty()) nm = a.name;
        if (!a.name.empty() && a.name != nm)
          fail(PSC_ERR_NAME, "dag spec: buffers \"" + nm + "\" and \"" + a.name + "\" are joined by an edge but named differently");
        if (a.output) rep = &a;
      }
      for (int32_t i : m) {
        const Arg &a = args[i];
        if (a.dtype != rep->dtype || a.rows != rep->rows || a.cols != rep->cols || a.view_of != rep->view_of ||
            a.row_off != rep->row_off || a.col_off != rep->col_off)
          fail(PSC_ERR_SHAPE, "dag spec: arguments (" + std::to_string(a.kernel) + "," + std::to_string(a.pos) + ") and (" +
                                  std::to_string(rep->kernel) + "," + std::to_string(rep->pos) +
                                  ") are one buffer but differ in type, shape or window");
      }
      if (nm.empty()) nm = "k" + std::to_string(rep->kernel) + "_a" + std::to_string(rep->pos);
      const bool is_root_name = root_by_name.count(nm) != 0;
      if (is_root_name) {
        const Root &r = roots[root_by_name[nm]];
        if (r.dtype != rep->dtype || r.rows != rep->rows || r.cols != rep->cols)
          fail(PSC_ERR_SHAPE, "dag spec: argument \"" + nm + "\" differs from its buffers entry in type or shape");
      } else {
        if (used_names.count(nm)) fail(PSC_ERR_NAME, "dag spec: buffer name \"" + nm + "\" is used twice");
        used_names.insert(nm);
        to_add.push_back({nm, rep});
      }
      for (int32_t i : m) arg_buf[i] = nm;
    }
    // lower onto the C ABI
    abi(psc_dag_create(&dag));
    for (const Root &r : roots) abi(psc_add_buffer(dag, r.name.c_str(), r.dtype, r.rows, r.cols, nullptr, 0, 0));
    for (const NewBuf &b : to_add)
      abi(psc_add_buffer(dag, b.name.c_str(), b.a->dtype, b.a->rows, b.a->cols,
                         b.a->view_of.empty() ? nullptr : b.a->view_of.c_str(), b.a->row_off, b.a->col_off));
    for (int32_t k = 0; k < nk; ++k) {
      std::vector<const char *> ins;
      const char *outb = nullptr;
      for (const auto &pa : arg_at[k]) {
        const Arg &a = args[pa.second];
        if (a.output) outb = arg_buf[pa.second].c_str();
        else ins.push_back(arg_buf[pa.second].c_str());
      }
      psc_kernel_params prm;
      std::memset(&prm, 0, sizeof(prm));
      prm.alpha = alpha[k];
      prm.alpha_set = 1;
      abi(psc_add_kernel(dag, kname[k].c_str(), kind[k], ins.data(), int32_t(ins.size()), &outb, 1, &prm, nullptr));
    }
    for (const Edge &e : edges)
      abi(psc_add_edge(dag, e.ki, arg_buf[arg_at[e.ki][e.br]].c_str(), e.kj, arg_buf[arg_at[e.kj][e.bs]].c_str()));
    // task components: sub-list i of tc is component i; kernels in no sub-list get components
    // after them, one each
    int32_t n_comp = 0;
    std::vector<int32_t> comp(nk, -1);
    if (const Json *tc = doc.get("tc")) {
      if (tc->type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: \"tc\" is not a list of lists");
      for (const Json &t : tc->arr) {
        if (t.type != Json::Arr) fail(PSC_ERR_ARG, "dag spec: \"tc\" is not a list of lists");
        for (const Json &x : t.arr) {
          const int64_t k = integer(x, sym, "tc");
          if (k < 0 || k >= nk) fail(PSC_ERR_ARG, "dag spec: tc names kernel " + std::to_string(k) + ", which does not exist");
          if (comp[k] >= 0) fail(PSC_ERR_ARG, "dag spec: kernel " + std::to_string(k) + " is in two task components");
          comp[k] = n_comp;
        }
        ++n_comp;
      }
    }
    for (int32_t k = 0; k < nk; ++k)
      if (comp[k] < 0) comp[k] = n_comp++;
    for (int32_t k = 0; k < nk; ++k) abi(psc_set_component(dag, k, comp[k]));
    // command queues: cq = {"gpu": n} or ["gpu:n", ...]
    int32_t queues = 0;
    if (const Json *cq = doc.get("cq")) {
      auto take = [&](const std::string &dev, int64_t n) {
        if (n < 0 || n > 64) fail(PSC_ERR_ARG, "dag spec: cq count out of range");
        if (dev == "gpu") queues = int32_t(n);
        else if (n > 0) fail(PSC_ERR_UNSUPPORTED, "dag spec: cq asks for queues on device \"" + dev + "\"; only gpu");
      };
      if (cq->type == Json::Obj) {
        for (const auto &kv : cq->obj) take(kv.first, integer(kv.second, sym, "cq"));
      } else if (cq->type == Json::Arr) {
        for (const Json &x : cq->arr) {
          const size_t colon = x.type == Json::Str ? x.str.find(':') : std::string::npos;
          if (colon == std::string::npos) fail(PSC_ERR_ARG, "dag spec: a cq entry is \"device:count\"");
          Json n;
          n.type = Json::Str;
          n.str = x.str.substr(colon + 1);
          take(x.str.substr(0, colon), integer(n, sym, "cq"));
        }
      } else {
        fail(PSC_ERR_ARG, "dag spec: \"cq\" is an object or a list");
      }
    }
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->n_kernels = nk;
      info->n_buffers = int32_t(roots.size() + to_add.size());
      info->n_edges = int32_t(edges.size());
      info->n_components = n_comp;
      info->gpu_queues = queues;
    }
    return dag;
  } catch (...) {
    if (dag) (void)psc_dag_destroy(dag);
    throw;
  }
}

}  // namespace psc
