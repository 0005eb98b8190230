// Reference evaluator for positive Datalog programs over uint32 relations.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; it exists so that tests, the smoke check and the CPU
// baseline leg of the benchmark can compare the GPU engine against a plain,
// slow, obviously correct evaluation.  It shares no code, header or table
// with the GPU engine.
//
// What it computes: the least fixpoint (minimal model) of a set of Horn
// clauses without function symbols over the extensional facts loaded
// (Section 2, "Datalog and RDF": rules H <- B1..Bn are applied until a fixed
// point is reached).  Two evaluation strategies are provided:
//
//  * semi-naive (Section 3, "Continuous Memory Layout" and "Schedule multiple
//    rules per iteration"): each relation is kept as full / delta / new; every
//    round evaluates all rules at once, with one body atom read from delta,
//    the new tuples are deduplicated and the difference against full becomes
//    the next delta, which is merged into full.  For the variant that reads
//    atom i from delta, atoms before i read full and atoms after i read
//    full minus delta, so that each derivation is produced by exactly one
//    variant.
//  * naive: full <- full U T_P(full) until nothing changes.
//
// Both produce the same round structure (round r derives exactly the facts
// whose shortest derivation has depth r), so their per-round delta sizes
// agree; tests use that, and independent brute-force checks, to pin this
// file.  Relations are sorted std::vector of fixed-width tuples; joins are
// index nested loops over sorted copies of a relation whose bound columns are
// moved to the front and searched with std::equal_range; the set difference
// and the merge use std::set_difference and std::merge.
//
// Rule syntax:  head(t, ...) :- atom(t, ...), ..., x != y.
// A term is a variable (identifier), an unsigned decimal constant, or `_`
// (a fresh variable at each occurrence).  `%` starts a comment.

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

namespace {

constexpr int kMaxArity = 3;
using Tup = std::array<uint32_t, kMaxArity>;   // unused trailing entries are 0

struct Term { bool is_const; uint32_t v; };    // constant value, or variable index
struct Atom { int rel; std::vector<Term> t; };
struct Rule {
  Atom head;
  std::vector<Atom> body;
  std::vector<std::pair<uint32_t, uint32_t>> neq;
  uint32_t nvars = 0;
};

struct Relation {
  std::string name;
  int arity = 0;
  bool idb = false;
  std::vector<Tup> full, delta, old;           // old = full minus delta
  std::vector<Tup> seed;                       // loaded facts (sorted, unique)
};

struct Ctx {
  std::vector<Relation> rels;
  std::map<std::string, int> by_name;
  std::vector<Rule> rules;
  std::vector<uint64_t> delta_sizes;           // sum over relations, per round
  double seconds = 0.0;
  std::string err;
  bool ran = false;
};

void sort_unique(std::vector<Tup>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}

// ------------------------------------------------------------------ parsing
struct Parser {
  const char* s;
  Ctx& c;
  std::map<std::string, uint32_t> vars;
  uint32_t nvars = 0;
  Parser(const char* text, Ctx& ctx) : s(text), c(ctx) {}

  void skip() {
    for (;;) {
      while (*s == ' ' || *s == '\t' || *s == '\n' || *s == '\r') ++s;
      if (*s == '%') { while (*s && *s != '\n') ++s; continue; }
      break;
    }
  }
  static bool id0(char ch) { return (ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || ch == '_'; }
  static bool id1(char ch) { return id0(ch) || (ch >= '0' && ch <= '9'); }
  std::string ident() {
    skip();
    if (!id0(*s)) throw std::runtime_error(std::string("expected identifier near: ") + std::string(s).substr(0, 20));
    const char* b = s;
    while (id1(*s)) ++s;
    return std::string(b, s);
  }
  void expect(const char* tok) {
    skip();
    size_t n = std::strlen(tok);
    if (std::strncmp(s, tok, n) != 0) throw std::runtime_error(std::string("expected '") + tok + "' near: " + std::string(s).substr(0, 20));
    s += n;
  }
  bool accept(const char* tok) {
    skip();
    size_t n = std::strlen(tok);
    if (std::strncmp(s, tok, n) == 0) { s += n; return true; }
    return false;
  }
  Term term() {
    skip();
    if (*s >= '0' && *s <= '9') {
      uint64_t v = 0;
      while (*s >= '0' && *s <= '9') { v = v * 10 + uint64_t(*s - '0'); ++s; if (v > 0xFFFFFFFEull) throw std::runtime_error("constant out of range"); }
      return Term{true, uint32_t(v)};
    }
    std::string name = ident();
    if (name == "_") return Term{false, nvars++};
    auto it = vars.find(name);
    if (it != vars.end()) return Term{false, it->second};
    vars[name] = nvars;
    return Term{false, nvars++};
  }
  int relation(const std::string& name, int arity) {
    auto it = c.by_name.find(name);
    if (it != c.by_name.end()) {
      if (c.rels[it->second].arity != arity) throw std::runtime_error("arity mismatch for " + name);
      return it->second;
    }
    if (arity < 1 || arity > kMaxArity) throw std::runtime_error("arity out of range for " + name);
    Relation r; r.name = name; r.arity = arity;
    c.rels.push_back(r);
    c.by_name[name] = int(c.rels.size()) - 1;
    return int(c.rels.size()) - 1;
  }
  Atom atom(const std::string& name) {
    Atom a;
    expect("(");
    a.t.push_back(term());
    while (accept(",")) a.t.push_back(term());
    expect(")");
    a.rel = relation(name, int(a.t.size()));
    return a;
  }
  void program() {
    for (;;) {
      skip();
      if (!*s) break;
      vars.clear(); nvars = 0;
      Rule r;
      r.head = atom(ident());
      expect(":-");
      do {
        skip();
        const char* save = s;
        std::string name = ident();
        skip();
        if (*s == '(') { r.body.push_back(atom(name)); continue; }
        s = save;
        Term x = term();
        expect("!=");
        Term y = term();
        if (x.is_const || y.is_const) throw std::runtime_error("!= takes two variables");
        r.neq.push_back({x.v, y.v});
      } while (accept(","));
      expect(".");
      r.nvars = nvars;
      // safety: every head and != variable must occur in a body atom
      std::vector<bool> pos(nvars, false);
      for (auto& b : r.body) for (auto& t : b.t) if (!t.is_const) pos[t.v] = true;
      for (auto& t : r.head.t) if (!t.is_const && !pos[t.v]) throw std::runtime_error("unsafe head variable");
      for (auto& p : r.neq) if (!pos[p.first] || !pos[p.second]) throw std::runtime_error("unsafe != variable");
      if (r.body.empty()) throw std::runtime_error("rule without body atoms");
      c.rels[r.head.rel].idb = true;
      c.rules.push_back(std::move(r));
    }
  }
};

// ------------------------------------------------------------------ joins
// A sorted copy of a relation whose columns are permuted so that the columns
// bound before the atom is visited come first; equal_range over that prefix
// yields exactly the tuples consistent with the current bindings.
struct Probe {
  int nkey = 0;
  std::array<int, kMaxArity> perm{};           // permuted position k holds column perm[k]
  const std::vector<Tup>* rows = nullptr;      // sorted permuted copy (or the source itself when nkey == 0)
};

// Sorted permuted copies of the sources read in one round, shared by every
// rule variant of the round (sources do not change within a round).
struct CopyCache {
  std::map<std::pair<const std::vector<Tup>*, int>, std::vector<Tup>> copies;
  const std::vector<Tup>* get(const std::vector<Tup>& src, const std::array<int, kMaxArity>& perm, int arity) {
    int sig = 0;
    for (int q = 0; q < arity; ++q) sig = sig * 4 + perm[q];
    auto key = std::make_pair(&src, sig * 4 + arity);
    auto it = copies.find(key);
    if (it != copies.end()) return &it->second;
    std::vector<Tup>& out = copies[key];
    out.resize(src.size());
    for (size_t j = 0; j < src.size(); ++j) {
      Tup t{};
      for (int q = 0; q < arity; ++q) t[q] = src[j][perm[q]];
      out[j] = t;
    }
    std::sort(out.begin(), out.end());
    return &out;
  }
};

enum ColKind { kConst, kBound, kFree, kRepeat };

struct AtomPlan {
  int arity = 0;
  std::array<ColKind, kMaxArity> kind{};
  std::array<uint32_t, kMaxArity> val{};       // constant value or variable index
  std::array<int, kMaxArity> rep_of{};         // kRepeat: column of the first occurrence
  std::vector<std::pair<uint32_t, uint32_t>> neq_here;  // != checks that become decidable here
  Probe probe;
};

// Atoms are visited in `order` (a permutation of the body positions); the
// join is commutative, so any order gives the same tuples.
struct BodyEval {
  const Rule& r;
  std::vector<AtomPlan> plans;
  std::vector<uint32_t> env;
  std::vector<Tup>* out;

  BodyEval(const Rule& rule, const std::vector<const std::vector<Tup>*>& src, const std::vector<size_t>& order,
           std::vector<Tup>* o, CopyCache& cache)
      : r(rule), plans(rule.body.size()), env(rule.nvars, 0), out(o) {
    std::vector<bool> bound(rule.nvars, false);
    std::vector<bool> neq_done(rule.neq.size(), false);
    for (size_t step = 0; step < rule.body.size(); ++step) {
      const size_t i = order[step];
      const Atom& a = rule.body[i];
      AtomPlan& p = plans[step];
      p.arity = int(a.t.size());
      std::vector<bool> bound_here = bound;
      for (int c = 0; c < p.arity; ++c) {
        const Term& t = a.t[c];
        p.val[c] = t.v;
        if (t.is_const) { p.kind[c] = kConst; continue; }
        if (bound[t.v]) { p.kind[c] = kBound; continue; }
        if (bound_here[t.v]) {
          p.kind[c] = kRepeat;
          for (int c2 = 0; c2 < c; ++c2)
            if (!a.t[c2].is_const && a.t[c2].v == t.v) { p.rep_of[c] = c2; break; }
          continue;
        }
        p.kind[c] = kFree;
        bound_here[t.v] = true;
      }
      bound = bound_here;
      for (size_t k = 0; k < rule.neq.size(); ++k)
        if (!neq_done[k] && bound[rule.neq[k].first] && bound[rule.neq[k].second]) {
          neq_done[k] = true;
          p.neq_here.push_back(rule.neq[k]);
        }
      // permuted, sorted copy of the source (an atom with no bound column is
      // scanned whole, in any order)
      int k = 0;
      for (int c = 0; c < p.arity; ++c) if (p.kind[c] == kConst || p.kind[c] == kBound) p.probe.perm[k++] = c;
      p.probe.nkey = k;
      for (int c = 0; c < p.arity; ++c) if (!(p.kind[c] == kConst || p.kind[c] == kBound)) p.probe.perm[k++] = c;
      if (p.probe.nkey == 0) {
        for (int c = 0; c < p.arity; ++c) p.probe.perm[c] = c;
        p.probe.rows = src[i];
      } else {
        p.probe.rows = cache.get(*src[i], p.probe.perm, p.arity);
      }
    }
  }

  void emit() {
    Tup h{};
    for (size_t c = 0; c < r.head.t.size(); ++c) {
      const Term& t = r.head.t[c];
      h[c] = t.is_const ? t.v : env[t.v];
    }
    out->push_back(h);
  }

  void visit(size_t i) {
    if (i == plans.size()) { emit(); return; }
    AtomPlan& p = plans[i];
    Tup key{};
    for (int q = 0; q < p.probe.nkey; ++q) {
      int c = p.probe.perm[q];
      key[q] = p.kind[c] == kConst ? p.val[c] : env[p.val[c]];
    }
    const int nk = p.probe.nkey;
    const std::vector<Tup>& rows = *p.probe.rows;
    auto lo = std::lower_bound(rows.begin(), rows.end(), key,
                               [nk](const Tup& a, const Tup& b) {
                                 for (int q = 0; q < nk; ++q) if (a[q] != b[q]) return a[q] < b[q];
                                 return false;
                               });
    for (auto it = lo; it != rows.end(); ++it) {
      bool same = true;
      for (int q = 0; q < nk; ++q) if ((*it)[q] != key[q]) { same = false; break; }
      if (!same) break;
      // un-permute the tuple
      Tup t{};
      for (int q = 0; q < p.arity; ++q) t[p.probe.perm[q]] = (*it)[q];
      bool ok = true;
      for (int c = 0; c < p.arity && ok; ++c) {
        if (p.kind[c] == kFree) env[p.val[c]] = t[c];
        else if (p.kind[c] == kRepeat) ok = (t[c] == t[p.rep_of[c]]);
      }
      for (auto& ne : p.neq_here) if (ok && env[ne.first] == env[ne.second]) ok = false;
      if (ok) visit(i + 1);
    }
  }
};

// Evaluate one rule variant: src[i] is the version atom i reads.  The atom
// reading the delta (first_atom) is visited first; after it, the first atom in
// written order that shares a variable with those already visited (or, if
// none does, the first remaining one).
void eval_rule(const Rule& r, const std::vector<const std::vector<Tup>*>& src, std::vector<Tup>& out,
               CopyCache& cache, size_t first_atom = 0) {
  std::vector<size_t> order{first_atom};
  std::vector<bool> used(r.body.size(), false), bound(r.nvars, false);
  used[first_atom] = true;
  for (auto& t : r.body[first_atom].t) if (!t.is_const) bound[t.v] = true;
  while (order.size() < r.body.size()) {
    size_t pick = r.body.size();
    for (size_t i = 0; i < r.body.size() && pick == r.body.size(); ++i) {
      if (used[i]) continue;
      for (auto& t : r.body[i].t) if (!t.is_const && bound[t.v]) { pick = i; break; }
    }
    for (size_t i = 0; i < r.body.size() && pick == r.body.size(); ++i) if (!used[i]) pick = i;
    order.push_back(pick);
    used[pick] = true;
    for (auto& t : r.body[pick].t) if (!t.is_const) bound[t.v] = true;
  }
  BodyEval e(r, src, order, &out, cache);
  e.visit(0);
}

// ------------------------------------------------------------------ fixpoint
void run(Ctx& c, bool naive) {
  for (auto& R : c.rels) {
    R.full = R.seed;
    R.delta.clear();
    R.old = R.full;
  }
  c.delta_sizes.clear();
  const size_t nrel = c.rels.size();
  auto t0 = std::chrono::steady_clock::now();
  bool first = true;
  for (;;) {
    std::vector<std::vector<Tup>> fresh(nrel);
    CopyCache cache;
    for (const Rule& r : c.rules) {
      std::vector<Tup>& out = fresh[r.head.rel];
      if (first || naive) {
        std::vector<const std::vector<Tup>*> src;
        for (auto& a : r.body) src.push_back(&c.rels[a.rel].full);
        eval_rule(r, src, out, cache);
        continue;
      }
      for (size_t i = 0; i < r.body.size(); ++i) {
        const Relation& Ri = c.rels[r.body[i].rel];
        if (!Ri.idb || Ri.delta.empty()) continue;
        std::vector<const std::vector<Tup>*> src;
        for (size_t j = 0; j < r.body.size(); ++j) {
          const Relation& Rj = c.rels[r.body[j].rel];
          src.push_back(j < i ? &Rj.full : (j == i ? &Rj.delta : &Rj.old));
        }
        eval_rule(r, src, out, cache, i);
      }
    }
    uint64_t total = 0;
    for (size_t k = 0; k < nrel; ++k) {
      Relation& R = c.rels[k];
      std::vector<Tup>& nw = fresh[k];
      sort_unique(nw);
      std::vector<Tup> d;
      std::set_difference(nw.begin(), nw.end(), R.full.begin(), R.full.end(), std::back_inserter(d));
      std::vector<Tup> merged;
      merged.reserve(R.full.size() + d.size());
      std::merge(R.full.begin(), R.full.end(), d.begin(), d.end(), std::back_inserter(merged));
      R.old.swap(R.full);            // old = full before this round's delta
      R.full.swap(merged);
      R.delta.swap(d);
      total += R.delta.size();
    }
    c.delta_sizes.push_back(total);
    first = false;
    if (total == 0) break;
  }
  c.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  c.ran = true;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

void* orc_create(void) { return new Ctx(); }
void orc_destroy(void* h) { delete static_cast<Ctx*>(h); }
const char* orc_error(void* h) { return static_cast<Ctx*>(h)->err.c_str(); }

int orc_program(void* h, const char* text) {
  Ctx& c = *static_cast<Ctx*>(h);
  try { Parser p(text, c); p.program(); return 0; }
  catch (const std::exception& e) { c.err = e.what(); return -1; }
}

// rows: n x arity, row-major
int orc_load(void* h, const char* name, uint32_t arity, const uint32_t* rows, uint64_t n) {
  Ctx& c = *static_cast<Ctx*>(h);
  try {
    int id;
    auto it = c.by_name.find(name);
    if (it == c.by_name.end()) {
      if (arity < 1 || arity > uint32_t(kMaxArity)) throw std::runtime_error("arity out of range");
      Relation r; r.name = name; r.arity = int(arity);
      c.rels.push_back(r);
      id = int(c.rels.size()) - 1;
      c.by_name[name] = id;
    } else {
      id = it->second;
      if (c.rels[id].arity != int(arity)) throw std::runtime_error("arity mismatch");
    }
    Relation& R = c.rels[id];
    for (uint64_t i = 0; i < n; ++i) {
      Tup t{};
      for (uint32_t q = 0; q < arity; ++q) t[q] = rows[i * arity + q];
      R.seed.push_back(t);
    }
    sort_unique(R.seed);
    return 0;
  } catch (const std::exception& e) { c.err = e.what(); return -1; }
}

int orc_run(void* h, int naive) {
  Ctx& c = *static_cast<Ctx*>(h);
  try { run(c, naive != 0); return 0; }
  catch (const std::exception& e) { c.err = e.what(); return -1; }
}

int64_t orc_size(void* h, const char* name) {
  Ctx& c = *static_cast<Ctx*>(h);
  auto it = c.by_name.find(name);
  if (it == c.by_name.end()) return -1;
  const Relation& R = c.rels[it->second];
  return int64_t(c.ran ? R.full.size() : R.seed.size());
}

int orc_export(void* h, const char* name, uint32_t* out, uint64_t cap) {
  Ctx& c = *static_cast<Ctx*>(h);
  auto it = c.by_name.find(name);
  if (it == c.by_name.end()) { c.err = "no such relation"; return -1; }
  const Relation& R = c.rels[it->second];
  const std::vector<Tup>& v = c.ran ? R.full : R.seed;
  if (cap < v.size()) { c.err = "capacity too small"; return -1; }
  for (size_t i = 0; i < v.size(); ++i)
    for (int q = 0; q < R.arity; ++q) out[i * R.arity + q] = v[i][q];
  return 0;
}

uint32_t orc_rounds(void* h) { return uint32_t(static_cast<Ctx*>(h)->delta_sizes.size()); }

int orc_delta_sizes(void* h, uint64_t* out, uint32_t cap) {
  Ctx& c = *static_cast<Ctx*>(h);
  if (cap < c.delta_sizes.size()) return -1;
  for (size_t i = 0; i < c.delta_sizes.size(); ++i) out[i] = c.delta_sizes[i];
  return 0;
}

double orc_seconds(void* h) { return static_cast<Ctx*>(h)->seconds; }

}  // extern "C"
