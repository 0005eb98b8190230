// Host runtime: relations, rule plans and the semi-naive round loop.
//
// A round (Section 3, "Schedule multiple rules per iteration") evaluates every
// rule variant at once -- one variant per body position that reads a delta --
// appending the head tuples of all variants of a relation to that relation's
// "new" buffer; then, per relation, the new tuples are radix-sorted, the
// difference against full is taken and the survivors are appended to the
// contiguous full relation, whose tail [d_begin, n_full) is the next delta.
//
// Sizes produced on the device (join outputs, deltas) stay on the device:
// kernels read them from counters, and buffers are sized ahead from known
// bounds.  A join whose output exceeds its buffer keeps counting, raises the
// overflow flag, and every later kernel of the round that would change state
// (sort, difference, merge, index rebuild) sees the flag and does nothing, so
// the host can grow the buffer and run the round again from the same state.
// The host reads the counters back once per round.
#include "engine.h"

#include <algorithm>
#include <array>
#include <cstdlib>
#include <cstring>
#include <functional>

namespace fv {

namespace {

u64 pow2_at_least(u64 x) {
  u64 p = 1;
  while (p < x) p <<= 1;
  return p;
}

u32 bits_for(u64 x) {   // number of bits to represent x (x >= 1)
  u32 b = 0;
  while (x) { ++b; x >>= 1; }
  return b;
}

}  // namespace

// Threads per block of a kernel class's launch over up to `rows` rows: the
// tuning's choice for that size bucket.
u32 Engine::block_for(int cls, u64 rows) const {
  const int b = rows <= (u64(1) << 16) ? 0 : rows <= (u64(1) << 20) ? 1 : rows <= (u64(1) << 24) ? 2 : 3;
  return 1u << tune_.block_log2[cls][b];
}

// ------------------------------------------------------------------ lifetime
Engine::Engine(const fv_options* opt) {
  if (opt) opt_ = *opt;
  if (opt_.tuning) tune_ = *opt_.tuning;
  opt_.tuning = nullptr;
  if (tune_.radix_bits != 11) tune_.radix_bits = 8;
  tune_.fuse_dedup = tune_.fuse_dedup ? 1 : 0;
  if (!(tune_.set_load >= 0.1f && tune_.set_load <= 0.75f)) tune_.set_load = 0.25f;
  if (!(tune_.index_load >= 0.1f && tune_.index_load <= 0.75f)) tune_.index_load = 0.5f;
  if (tune_.max_blocks < 256 || tune_.max_blocks > 8192) tune_.max_blocks = 2048;
  tune_.index_rebuild = tune_.index_rebuild ? 1 : 0;
  if (tune_.index_sort > 2) tune_.index_sort = 0;
  tune_.lookahead = tune_.lookahead ? 1 : 0;
  if (tune_.dedup_ranges > 2) tune_.dedup_ranges = 0;
  for (auto& cls : tune_.block_log2)
    for (auto& l : cls)
      if (l != 7 && l != 9) l = 8;
  if (opt_.dev_alloc && !opt_.dev_free) throw Error(FV_EINVAL, "dev_alloc given without dev_free");
  stream_ = static_cast<hipStream_t>(opt_.stream);
  host_mode_ = (opt_.flags & FV_HOST) != 0;
  if (host_mode_) {
    if (opt_.flags & (FV_LEARNED | FV_GRAPH | FV_LOG_JOINS))
      throw Error(FV_EINVAL, "FV_HOST runs the plain engine only (no FV_LEARNED, FV_GRAPH or FV_LOG_JOINS)");
    opt_.flags &= ~u32(FV_TRACE);
    host_threads_ = host_threads();
  }
  trace_ = (opt_.flags & FV_TRACE) != 0;
  if (trace_) {   // the constant-rate clock the kernels stamp (kHz)
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      wall_khz_ = double(khz);
    (void)hipGetLastError();
  }
  // per-kernel event timing needs the kernels launched one by one
  use_graph_ = !trace_ && (opt_.flags & FV_GRAPH);
  learned_ = (opt_.flags & FV_LEARNED) != 0;
  log_joins_ = learned_ || (opt_.flags & FV_LOG_JOINS) != 0;
  if (learned_) {
    if (!opt_.predictor) throw Error(FV_EINVAL, "FV_LEARNED needs fv_options.predictor");
    predictor_.assign(opt_.predictor, opt_.predictor + kMlpParams);
  }
  opt_.predictor = nullptr;
  if (opt_.trace_only) trace_only_ = opt_.trace_only;
  opt_.trace_only = nullptr;
  // Test hooks (fault injection for the redo paths), read once per context:
  // FV_TEST_FAIL_ROUNDS="3,5" makes the 3rd and 5th enqueued rounds fail once
  // as if a join had overflowed; FV_TEST_SMALL_CAPS=1 starts every new-tuple
  // and intermediate buffer at 256 rows, so that the first rounds overflow
  // and grow.
  if (const char* f = std::getenv("FV_TEST_FAIL_ROUNDS")) {
    for (const char* q = f; *q;) {
      char* end = nullptr;
      const unsigned long v = std::strtoul(q, &end, 10);
      if (end == q) { ++q; continue; }
      fail_rounds_.insert(u64(v));
      q = end;
    }
  }
  if (const char* c = std::getenv("FV_TEST_SMALL_CAPS")) small_caps_ = std::atoi(c) != 0;
}

Engine::~Engine() {
  // best effort: wait for queued work, then free everything
  if (touched_device_) (void)hipStreamSynchronize(stream_);
  drop_graph();
  for (auto& R : rels_) {
    for (int c = 0; c < 3; ++c) { release(R.stage[c]); release(R.col[c]); }
    release(R.newk); release(R.newk2); release(R.set); release(R.sfull); release(R.sfull2);
  }
  for (auto& ix : indices_) {
    release(ix.table); release(ix.perm); release(ix.pcap); release(ix.dcnt); release(ix.wl);
  }
  release(moves_);
  for (auto& I : inters_) for (auto& b : I.col) release(b);
  flags_dev_ = Buf{};   // a view into ctr_dev_
  release(ctr_dev_); release(ticket_dev_); release(hist_dev_); release(maxv_dev_); release(dict_);
  release(stamps_dev_);
  release(m_row_); release(m_start_); release(m_off_);
  release(st_a_); release(st_b_); release(st_sort_);
  release(mdiff_);
  release(ixk_a_); release(ixk_b_);
  for (auto& sk : sketches_) release(sk.regs);
  release(predictor_dev_); release(pspec_init_dev_); release(pspec_delta_dev_);
  for (int i = 0; i < 2; ++i) {   // ctr_host_ and flags_host_ point into these
    if (rb_host_[i]) (void)hipHostFree(rb_host_[i]);
    if (rb_ev_[i]) (void)hipEventDestroy(rb_ev_[i]);
  }
  for (auto e : ev_pool_) (void)hipEventDestroy(e);
  for (auto& p : pending_) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
}

// ------------------------------------------------------------------ memory
Buf Engine::alloc(size_t bytes) {
  touched_device_ = true;
  ++n_allocs_;
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  if (opt_.dev_alloc) {
    p = opt_.dev_alloc(bytes, opt_.stream, opt_.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  host_time("host_alloc", t0);
  if (!p) {
    terminal = true;
    throw Error(FV_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  Buf b;
  b.p = p;
  b.bytes = bytes;
  return b;
}

void Engine::release(Buf& b) {
  if (b.p) {
    if (opt_.dev_free) opt_.dev_free(b.p, opt_.stream, opt_.user);
    else (void)hipFree(b.p);
  }
  b = Buf{};
}

void Engine::grow(Buf& b, size_t bytes, size_t keep_bytes) {
  if (b.p && b.bytes >= bytes) return;
  Buf nb = alloc(bytes);
  if (b.p && keep_bytes)
    hip(hipMemcpyAsync(nb.p, b.p, std::min(keep_bytes, b.bytes), hipMemcpyDeviceToDevice, stream_), "grow copy");
  release(b);
  b = nb;
}

void Engine::hip(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    terminal = true;
    throw Error(FV_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  }
}

void Engine::launched(int rc, const char* what) { hip(static_cast<hipError_t>(rc), what); }

void Engine::sync() { hip(hipStreamSynchronize(stream_), "stream synchronize"); }

// A phase starts by advancing the device epoch base; every look-back launch in
// the phase takes base + a distinct offset.  After 4000 phases (the 22-bit
// epoch would wrap after 4096) the status arrays and the base are cleared.
void Engine::begin_phase() {
  if (phases_ + 2 >= (kEpochMask + 1) / kEpochStride - 96) {
    if (st_a_.p) launched(launch_fill_u64(st_a_.as<u64>(), st_a_.bytes / 8, 0, stream_), "clear status");
    if (st_b_.p) launched(launch_fill_u64(st_b_.as<u64>(), st_b_.bytes / 8, 0, stream_), "clear status");
    if (st_sort_.p) launched(launch_fill_u64(st_sort_.as<u64>(), st_sort_.bytes / 8, 0, stream_), "clear status");
    launched(launch_fill_u32(epoch_base(), 1, 0u, stream_), "epoch reset");
    phases_ = 0;
  }
  // a new phase starts with the overflow and set-full flags down: kernels that
  // rebuild state before the next round (index builds) skip their work while
  // the flag of a failed round is still up
  launched(launch_round_prologue(nullptr, 0, flags_dev_.p ? flags_dev_.as<u32>() : nullptr, nullptr, 0, epoch_base(),
                                 stream_),
           "epoch advance");
  ++phases_;
  epoch_off_ = 1;
}

u32 Engine::next_epoch() {
  if (epoch_off_ >= kEpochStride) throw Error(FV_ENOTSUP, "too many look-back launches in one round");
  return epoch_off_++;
}

// ------------------------------------------------------------------ relations and rules
u32 Engine::relation_create(const char* name, u32 arity) {
  if (!name || !*name) throw Error(FV_EINVAL, "relation name is empty");
  if (ran_) throw Error(FV_ESTATE, "relations cannot be added after the fixpoint ran");
  if (arity < 1 || arity > 3) throw Error(FV_EARITY, "arity must be 1..3");
  if (by_name_.count(name)) throw Error(FV_EINVAL, std::string("relation exists: ") + name);
  Relation R;
  R.name = name;
  R.arity = arity;
  rels_.push_back(R);
  const u32 id = u32(rels_.size() - 1);
  by_name_[name] = id;
  return id;
}

u32 Engine::relation_find(const char* name) const {
  if (!name) throw Error(FV_EINVAL, "null name");
  auto it = by_name_.find(name);
  if (it == by_name_.end()) throw Error(FV_EINVAL, std::string("no relation named ") + name);
  return it->second;
}

void Engine::load_columns(u32 rel, const u32* const* cols, u64 n, bool on_device) {
  if (rel >= rels_.size()) throw Error(FV_EINVAL, "bad relation handle");
  if (ran_) throw Error(FV_ESTATE, "facts cannot be loaded after the fixpoint ran");
  if (n == 0) return;
  if (!cols) throw Error(FV_EINVAL, "null column array");
  Relation& R = rels_[rel];
  for (u32 c = 0; c < R.arity; ++c)
    if (!cols[c]) throw Error(FV_EINVAL, "null column pointer");
  if (host_mode_) { host_load(rel, cols, n, on_device); return; }
  if (!maxv_dev_.p) maxv_dev_ = alloc(64);
  if (R.staged + n > R.stage_cap) {
    const u64 cap = std::max<u64>(R.staged + n, R.stage_cap * 2);
    for (u32 c = 0; c < R.arity; ++c) grow(R.stage[c], cap * 4, R.staged * 4);
    R.stage_cap = cap;
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  u32* mx = maxv_dev_.as<u32>();
  launched(launch_fill_u32(mx, 4, 0u, stream_), "fill");
  for (u32 c = 0; c < R.arity; ++c) {
    u32* dst = R.stage[c].as<u32>() + R.staged;
    hip(hipMemcpyAsync(dst, cols[c], n * 4, kind, stream_), "load copy");
    launched(launch_colmax(dst, n, mx + c, stream_), "colmax");
  }
  u32 host_max[4] = {0, 0, 0, 0};
  hip(hipMemcpyAsync(host_max, mx, 16, hipMemcpyDeviceToHost, stream_), "max readback");
  sync();
  for (u32 c = 0; c < R.arity; ++c)
    if (host_max[c] == 0xFFFFFFFFu) throw Error(FV_ERESERVED, "value 0xFFFFFFFF is reserved");
  for (u32 c = 0; c < R.arity; ++c) {
    R.maxv[c] = std::max(R.maxv[c], host_max[c]);
    R.lmax[c] = std::max(R.lmax[c], host_max[c]);
  }
  R.staged += n;
  R.has_rows = true;
}

void Engine::add_rule(const fv_rule& r) {
  if (ran_) throw Error(FV_ESTATE, "rules cannot be added after the fixpoint ran");
  auto conv = [&](const fv_atom& a) {
    if (a.rel >= rels_.size()) throw Error(FV_EINVAL, "bad relation handle in rule");
    if (a.arity != rels_[a.rel].arity) throw Error(FV_EARITY, "atom arity differs from relation " + rels_[a.rel].name);
    if (!a.terms) throw Error(FV_EINVAL, "null terms");
    AtomR o;
    o.rel = a.rel;
    for (u32 i = 0; i < a.arity; ++i) {
      const fv_term& t = a.terms[i];
      if (t.is_const) {
        if (t.value == 0xFFFFFFFFu) throw Error(FV_ERESERVED, "constant 0xFFFFFFFF is reserved");
      } else if (t.value >= kMaxVars) {
        throw Error(FV_EINVAL, "variable index above 15");
      }
      o.t.push_back(Term{t.value, t.is_const != 0});
    }
    return o;
  };
  if (r.n_body < 1 || r.n_body > kMaxBody) throw Error(FV_EINVAL, "a rule needs 1..8 body atoms");
  if (r.n_neq > kMaxNeq) throw Error(FV_EINVAL, "at most 8 != constraints");
  if (!r.body) throw Error(FV_EINVAL, "null body");
  RuleR rr;
  rr.head = conv(r.head);
  for (u32 i = 0; i < r.n_body; ++i) rr.body.push_back(conv(r.body[i]));
  bool pos[kMaxVars] = {};
  for (auto& a : rr.body)
    for (auto& t : a.t)
      if (!t.is_const) pos[t.value] = true;
  for (auto& t : rr.head.t)
    if (!t.is_const && !pos[t.value]) throw Error(FV_EUNSAFE, "head variable not bound by the body");
  if (r.n_neq && !r.neq) throw Error(FV_EINVAL, "null neq");
  for (u32 i = 0; i < r.n_neq; ++i) {
    const u32 a = r.neq[2 * i], b = r.neq[2 * i + 1];
    if (a >= kMaxVars || b >= kMaxVars) throw Error(FV_EINVAL, "variable index above 15");
    if (!pos[a] || !pos[b]) throw Error(FV_EUNSAFE, "!= variable not bound by the body");
    rr.neq.push_back({a, b});
  }
  rules_.push_back(rr);
}

u64 Engine::relation_size(u32 rel) const {
  if (rel >= rels_.size()) throw Error(FV_EINVAL, "bad relation handle");
  return ran_ ? rels_[rel].n_full : rels_[rel].staged;
}

// ------------------------------------------------------------------ domain analysis
// Datalog without function symbols creates no values: a head column can only
// hold constants of the rule or values of a body column its variable occurs
// in, so its maximum is bounded by the smallest maximum over those columns.
// The bounds give each column a bit width for the packed tuple key; false if
// some relation's key would need more than 64 bits.
bool Engine::domain_analysis() {
  for (auto& r : rules_) rels_[r.head.rel].idb = true;
  for (bool changed = true; changed;) {
    changed = false;
    for (auto& r : rules_) {
      Relation& H = rels_[r.head.rel];
      for (u32 c = 0; c < H.arity; ++c) {
        const Term& t = r.head.t[c];
        u32 m;
        if (t.is_const) {
          m = t.value;
        } else {
          m = 0xFFFFFFFEu;
          for (auto& a : r.body)
            for (u32 k = 0; k < a.t.size(); ++k)
              if (!a.t[k].is_const && a.t[k].value == t.value) m = std::min(m, rels_[a.rel].maxv[k]);
        }
        if (m > H.maxv[c]) { H.maxv[c] = m; changed = true; }
      }
    }
  }
  refine_bounds();
  bool fits = true;
  for (auto& R : rels_) {
    // a column needs bits(max) bits; a packed key can only equal the
    // all-ones empty-slot sentinel if it fills all 64 bits with every field
    // at its all-ones value, so in that case each field gets bits(max + 1)
    // (which keeps it strictly below all-ones)
    R.bits = 0;
    for (u32 c = 0; c < R.arity; ++c) {
      R.width[c] = std::max<u32>(1, bits_for(R.maxv[c]));
      R.bits += R.width[c];
    }
    if (R.bits >= 64) {
      R.bits = 0;
      for (u32 c = 0; c < R.arity; ++c) {
        R.width[c] = bits_for(u64(R.maxv[c]) + 1);
        R.bits += R.width[c];
      }
    }
    if (R.bits > 64) { fits = false; continue; }
    u32 s = 0;
    for (int c = int(R.arity) - 1; c >= 0; --c) { R.shift[c] = s; s += R.width[c]; }
    R.set32 = R.bits <= 32;
  }
  return fits;
}

// Tighter bounds from the rules' constant conditions.  The bound above takes
// a head variable's maximum over whole body columns; but a body atom with
// constants reads only the rows that match them, and rules often fill a
// column with values drawn from such rows (RDFS: the property column of a
// derived triple filled from subPropertyOf rows, whose objects are
// properties).  Every relation gets one interval per column for each set of
// constant positions a body atom over it has, and one for all of its rows.
// The facts give the first intervals (one pass over them); a rule adds to a
// condition set of its head when its head row can meet the conditions (a
// head constant equal to the value, or a variable whose interval holds it,
// which is then fixed to it), each head column bounded by its constant or by
// the intersection of the intervals of the body columns its variable reads,
// under those atoms' conditions.  Intervals only widen, to endpoints taken
// from the facts and the constants, so the iteration ends.  A column's bound
// becomes the smaller of the one above and its all-rows interval's maximum.
void Engine::refine_bounds() {
  struct Ival {
    u32 lo = 1, hi = 0;   // empty
    bool empty() const { return lo > hi; }
  };
  const u32 nrel = u32(rels_.size());
  std::vector<std::vector<CondSet>> sets(nrel, std::vector<CondSet>(1, CondSet{}));
  std::vector<std::vector<u32>> atom_set(rules_.size());
  bool any_const = false;
  for (size_t ri = 0; ri < rules_.size(); ++ri)
    for (auto& a : rules_[ri].body) {
      CondSet q{};
      for (u32 k = 0; k < a.t.size(); ++k)
        if (a.t[k].is_const) {
          q.col[q.n] = k;
          q.val[q.n] = a.t[k].value;
          ++q.n;
        }
      any_const = any_const || q.n > 0;
      auto& v = sets[a.rel];
      u32 at = 0;
      while (at < v.size() && !(v[at].n == q.n && std::equal(q.col, q.col + q.n, v[at].col) &&
                                std::equal(q.val, q.val + q.n, v[at].val)))
        ++at;
      if (at == v.size()) v.push_back(q);
      atom_set[ri].push_back(at);
    }
  if (!any_const) return;
  std::vector<std::vector<std::array<Ival, 3>>> iv(nrel);
  for (u32 r = 0; r < nrel; ++r) {
    const Relation& R = rels_[r];
    iv[r].assign(sets[r].size(), std::array<Ival, 3>{});
    if (!R.has_rows || R.staged == 0) continue;
    std::vector<u32> out(kCondSets * 8);
    for (u32 q0 = 0; q0 < sets[r].size(); q0 += kCondSets) {
      const u32 nq = std::min<u32>(kCondSets, u32(sets[r].size()) - q0);
      if (host_mode_) host_fact_bounds(r, &sets[r][q0], nq, out.data());
      else fact_bounds(r, &sets[r][q0], nq, out.data());
      for (u32 q = 0; q < nq; ++q) {
        if (!out[q * 8 + 6]) continue;
        for (u32 c = 0; c < R.arity; ++c) iv[r][q0 + q][c] = Ival{out[q * 8 + c], out[q * 8 + 3 + c]};
      }
    }
  }
  bool settled = false;
  for (int it = 0; it < 100000 && !settled; ++it) {
    settled = true;
    for (size_t ri = 0; ri < rules_.size(); ++ri) {
      const RuleR& rule = rules_[ri];
      Ival var[kMaxVars];
      for (auto& v : var) v = Ival{0, 0xFFFFFFFEu};
      bool feasible = true;
      for (size_t b = 0; b < rule.body.size() && feasible; ++b) {
        const AtomR& a = rule.body[b];
        const auto& I = iv[a.rel][atom_set[ri][b]];
        if (I[0].empty()) { feasible = false; break; }   // no row can match the atom
        for (u32 k = 0; k < a.t.size(); ++k) {
          if (a.t[k].is_const) continue;
          Ival& x = var[a.t[k].value];
          x.lo = std::max(x.lo, I[k].lo);
          x.hi = std::min(x.hi, I[k].hi);
          if (x.empty()) feasible = false;
        }
      }
      if (!feasible) continue;
      const u32 h = rule.head.rel;
      for (u32 si = 0; si < sets[h].size(); ++si) {
        const CondSet& q = sets[h][si];
        Ival loc[kMaxVars];
        std::copy(var, var + kMaxVars, loc);
        bool meets = true;
        for (u32 i = 0; i < q.n && meets; ++i) {
          const Term& t = rule.head.t[q.col[i]];
          if (t.is_const) {
            meets = t.value == q.val[i];
          } else {
            Ival& x = loc[t.value];
            meets = q.val[i] >= x.lo && q.val[i] <= x.hi;
            x = Ival{q.val[i], q.val[i]};
          }
        }
        if (!meets) continue;
        for (u32 c = 0; c < rels_[h].arity; ++c) {
          const Term& t = rule.head.t[c];
          const Ival v = t.is_const ? Ival{t.value, t.value} : loc[t.value];
          Ival& d = iv[h][si][c];
          if (d.empty()) {
            d = v;
            settled = false;
          } else {
            if (v.lo < d.lo) { d.lo = v.lo; settled = false; }
            if (v.hi > d.hi) { d.hi = v.hi; settled = false; }
          }
        }
      }
    }
  }
  if (!settled) return;   // (not reached: the endpoints are finitely many)
  for (u32 r = 0; r < nrel; ++r)
    for (u32 c = 0; c < rels_[r].arity; ++c)
      if (!iv[r][0][c].empty()) rels_[r].maxv[c] = std::min(rels_[r].maxv[c], iv[r][0][c].hi);
}

void Engine::fact_bounds(u32 rel, const CondSet* q, u32 nq, u32* out) {
  const Relation& R = rels_[rel];
  Buf d = alloc(kCondSets * 8 * 4);
  try {
    CondBoundsArgs a{};
    for (u32 c = 0; c < R.arity; ++c) a.col[c] = R.stage[c].as<u32>();
    a.arity = R.arity;
    a.n_rows = R.staged;
    a.nq = nq;
    for (u32 i = 0; i < nq; ++i) a.q[i] = q[i];
    a.out = d.as<u32>();
    launched(launch_cond_bounds(a, stream_), "bounds launch");
    hip(hipMemcpyAsync(out, d.p, size_t(nq) * 8 * 4, hipMemcpyDeviceToHost, stream_), "bounds readback");
    sync();
  } catch (...) {
    release(d);
    throw;
  }
  release(d);
}

// Relations whose packed tuples need more than 64 bits (three columns of
// large ids): values are only compared for equality and no rule creates new
// ones, so every value of the loaded facts and of the rules' constants is
// replaced by its rank among the distinct ones (order kept: exports map the
// ranks back after sorting).  Widths then follow the number of distinct
// values rather than their magnitude.
void Engine::fit_packing() {
  auto widest = [&]() {
    const Relation* w = &rels_[0];
    for (auto& R : rels_) if (R.bits > w->bits) w = &R;
    return w;
  };
  if (rels_.empty() || domain_analysis()) return;
  if (!allow_compaction_) {
    const Relation* w = widest();
    throw Error(FV_ENOTSUP, "relation " + w->name + " needs " + std::to_string(w->bits) + " bits per packed tuple");
  }
  if (host_mode_) host_compact_values();
  else compact_values();
  compacted_ = true;
  auto rank = [&](u32 v) {
    return u32(std::lower_bound(dict_host_.begin(), dict_host_.end(), v) - dict_host_.begin());
  };
  for (auto& r : rules_) {
    for (auto& t : r.head.t) if (t.is_const) t.value = rank(t.value);
    for (auto& a : r.body) for (auto& t : a.t) if (t.is_const) t.value = rank(t.value);
  }
  for (auto& R : rels_)
    for (u32 c = 0; c < R.arity; ++c) R.maxv[c] = R.has_rows ? rank(R.lmax[c]) : 0;
  if (!domain_analysis()) {
    const Relation* w = widest();
    throw Error(FV_ENOTSUP, "relation " + w->name + " needs " + std::to_string(w->bits) +
                                " bits per packed tuple even with its values renumbered densely (" +
                                std::to_string(dict_host_.size()) + " distinct values)");
  }
}

// Sorted distinct values of every loaded column and rule constant (radix sort
// of the values, then the heads of equal runs), and every loaded column
// rewritten as ranks.  Runs before the control buffers exist, so the sort
// gets look-back words, ticket and histogram of its own.
void Engine::compact_values() {
  std::vector<u64> consts;
  for (auto& r : rules_) {
    for (auto& t : r.head.t) if (t.is_const) consts.push_back(t.value);
    for (auto& a : r.body) for (auto& t : a.t) if (t.is_const) consts.push_back(t.value);
  }
  u64 total = consts.size();
  for (auto& R : rels_) total += R.staged * R.arity;
  if (total == 0) total = 1;
  const u64 stiles = (total + kSortTile - 1) / kSortTile + 1;
  Buf a, b, ctl, hist, status, tiles, d;
  auto release_all = [&]() {
    release(a); release(b); release(ctl); release(hist); release(status); release(tiles);
  };
  try {
    a = alloc(total * 8);
    b = alloc(total * 8);
    ctl = alloc(64);
    hist = alloc(kHistWords * 4);
    status = alloc(stiles * kMaxRadix * 8);
    tiles = alloc((dict_tiles(total) + 1) * 8);
    d = alloc(total * 4);
    launched(launch_fill_u32(ctl.as<u32>(), 16, 0u, stream_), "fill");
    launched(launch_fill_u64(status.as<u64>(), stiles * kMaxRadix, 0, stream_), "fill");
    launched(launch_fill_u64(a.as<u64>(), total, 0, stream_), "fill");
    u64 off = 0;
    for (auto& R : rels_)
      for (u32 c = 0; c < R.arity && R.staged; ++c) {
        const u32* in[1] = {R.stage[c].as<u32>()};
        const u32 sh[1] = {0};
        launched(launch_pack(in, 1, sh, R.staged, a.as<u64>() + off, stream_), "pack launch");
        off += R.staged;
      }
    if (!consts.empty())
      hip(hipMemcpyAsync(a.as<u64>() + off, consts.data(), consts.size() * 8, hipMemcpyHostToDevice, stream_),
          "constant copy");
    SortParams sp{};
    sp.a = a.as<u64>();
    sp.b = b.as<u64>();
    sp.n_const = total;
    sp.cap = total;
    sp.bits = 32;
    sp.digit_bits = 8;
    sp.max_blocks = tune_.max_blocks;
    sp.hist = hist.as<u32>();
    sp.status = status.as<u64>();
    sp.ticket = ctl.as<u32>();
    sp.epoch_base = ctl.as<u32>() + 8;
    launched(launch_rs_hist(sp, stream_), "hist launch");
    u64* src = sp.a;
    u64* dst = sp.b;
    for (u32 pass = 0; pass < sort_passes(32, 8); ++pass) {
      launched(launch_rs_pass(sp, pass, src, dst, pass + 1, stream_), "sort pass launch");
      std::swap(src, dst);
    }
    const u64 nt = dict_tiles(total);
    launched(launch_dict_unique(src, total, tiles.as<u64>(), d.as<u32>(), tiles.as<u64>() + nt, stream_),
             "dictionary launch");
    u64 nd = 0;
    hip(hipMemcpyAsync(&nd, tiles.as<u64>() + nt, 8, hipMemcpyDeviceToHost, stream_), "count readback");
    sync();
    dict_host_.resize(nd);
    hip(hipMemcpyAsync(dict_host_.data(), d.p, nd * 4, hipMemcpyDeviceToHost, stream_), "dictionary readback");
    for (auto& R : rels_)
      for (u32 c = 0; c < R.arity && R.staged; ++c)
        launched(launch_dict_remap(R.stage[c].as<u32>(), R.staged, d.as<u32>(), nd, stream_), "remap launch");
    sync();
  } catch (...) {
    release_all();
    release(d);
    throw;
  }
  release_all();
  dict_ = d;
}

// Exported rows hold ranks when the values were compacted: map them back.
void Engine::map_back(u32* const* cols, u32 arity, u64 n, bool on_device) {
  if (!compacted_ || n == 0) return;
  if (on_device) {
    for (u32 c = 0; c < arity; ++c) launched(launch_dict_gather(cols[c], n, dict_.as<u32>(), stream_), "gather launch");
    sync();
  } else {
    for (u32 c = 0; c < arity; ++c)
      for (u64 i = 0; i < n; ++i) cols[c][i] = dict_host_[cols[c][i]];
  }
}

// ------------------------------------------------------------------ planning
// The index of `rel` on key columns `keycol` over the rows that satisfy the
// filters col[fcol[i]] == fval[i] (i < nfilt; filters given in column order),
// shared by every join that asks for the same one.
u32 Engine::get_index(u32 rel, u32 nkey, const u32* keycol, u32 nfilt, const u32* fcol, const u32* fval) {
  for (u32 i = 0; i < indices_.size(); ++i) {
    const Index& ix = indices_[i];
    if (ix.rel != rel || ix.nkey != nkey || ix.keycol[0] != keycol[0] || (nkey > 1 && ix.keycol[1] != keycol[1]) ||
        ix.nfilt != nfilt)
      continue;
    bool same = true;
    for (u32 f = 0; f < nfilt; ++f) same = same && ix.fcol[f] == fcol[f] && ix.fval[f] == fval[f];
    if (same) return i;
  }
  Index ix;
  ix.rel = rel;
  ix.nkey = nkey;
  ix.keycol[0] = keycol[0];
  ix.keycol[1] = nkey > 1 ? keycol[1] : 0;
  ix.nfilt = nfilt;
  for (u32 f = 0; f < nfilt; ++f) { ix.fcol[f] = fcol[f]; ix.fval[f] = fval[f]; }
  indices_.push_back(ix);
  return u32(indices_.size() - 1);
}

Plan Engine::plan_rule(u32 ri, int dpos, int second) {
  const RuleR& r = rules_[ri];
  const u32 nb = u32(r.body.size());
  std::vector<bool> used(nb, false), bound(kMaxVars, false);
  std::vector<u32> order;
  u32 first = 0;
  if (dpos >= 0) {
    first = u32(dpos);
  } else {
    u64 best = ~0ull;
    for (u32 i = 0; i < nb; ++i) {
      const Relation& R = rels_[r.body[i].rel];
      if (R.staged < best) { best = R.staged; first = i; }
    }
  }
  order.push_back(first);
  used[first] = true;
  for (auto& t : r.body[first].t)
    if (!t.is_const) bound[t.value] = true;
  // Next atom, most bound first: one connected to what is bound (or with no
  // variable left to bind), then the fewest variables it newly binds (an atom
  // bound in every position is a semi-join and can only shrink the result),
  // then the most shared variables, the most constants, EDB before IDB.
  // (`second`, when given, names the atom the first join reads instead)
  while (order.size() < nb) {
    int best = -1;
    long best_score = -1;
    for (u32 i = 0; i < nb; ++i) {
      if (used[i]) continue;
      if (second >= 0 && order.size() == 1) {
        if (int(i) == second) best = int(i);
        continue;
      }
      int shared = 0, consts = 0, fresh = 0;
      std::vector<bool> seen(kMaxVars, false);
      for (auto& t : r.body[i].t) {
        if (t.is_const) { ++consts; continue; }
        if (seen[t.value]) continue;
        seen[t.value] = true;
        if (bound[t.value]) ++shared;
        else ++fresh;
      }
      const bool connected = shared > 0 || fresh == 0;
      const long score = (connected ? 1L << 24 : 0) + long(kMaxCols + 1 - fresh) * 4096 + shared * 64 + consts * 4 +
                         (rels_[r.body[i].rel].idb ? 0 : 1);
      if (score > best_score) { best_score = score; best = int(i); }
    }
    order.push_back(u32(best));
    used[best] = true;
    for (auto& t : r.body[best].t)
      if (!t.is_const) bound[t.value] = true;
  }

  Plan p;
  p.rule = ri;
  p.delta_pos = dpos;
  p.src_rel = r.body[first].rel;
  p.src_delta = dpos >= 0;
  p.second = nb > 1 ? order[1] : 0;

  // which variables are still needed after body position k of `order`
  auto needed_after = [&](u32 k, const std::vector<bool>& neq_done) {
    std::vector<bool> need(kMaxVars, false);
    for (u32 j = k + 1; j < nb; ++j)
      for (auto& t : r.body[order[j]].t)
        if (!t.is_const) need[t.value] = true;
    for (auto& t : r.head.t)
      if (!t.is_const) need[t.value] = true;
    for (u32 q = 0; q < r.neq.size(); ++q)
      if (!neq_done[q]) { need[r.neq[q].first] = true; need[r.neq[q].second] = true; }
    return need;
  };

  // schema of the probe side: variable -> probe column
  std::vector<int> schema(kMaxVars, -1);
  std::vector<bool> neq_done(r.neq.size(), false);
  std::vector<Filter> pf;
  {
    const AtomR& a0 = r.body[first];
    for (u32 c = 0; c < a0.t.size(); ++c) {
      const Term& t = a0.t[c];
      if (t.is_const) pf.push_back(Filter{Src{kSrcProbe, c}, Src{kSrcConst, t.value}, kEq});
      else if (schema[t.value] >= 0) pf.push_back(Filter{Src{kSrcProbe, c}, Src{kSrcProbe, u32(schema[t.value])}, kEq});
      else schema[t.value] = int(c);
    }
    for (u32 q = 0; q < r.neq.size(); ++q) {
      const int a = schema[r.neq[q].first], b = schema[r.neq[q].second];
      if (a >= 0 && b >= 0) {
        pf.push_back(Filter{Src{kSrcProbe, u32(a)}, Src{kSrcProbe, u32(b)}, kNe});
        neq_done[q] = true;
      }
    }
  }
  if (pf.size() > size_t(kMaxFilters)) throw Error(FV_ENOTSUP, "too many filters on one atom");

  auto head_out = [&](const std::vector<Src>& var_src) {
    std::vector<Src> out;
    for (auto& t : r.head.t) out.push_back(t.is_const ? Src{kSrcConst, t.value} : var_src[t.value]);
    return out;
  };

  if (nb == 1) {
    Step s;
    s.select_only = true;
    s.pf = pf;
    std::vector<Src> vs(kMaxVars, Src{kSrcConst, 0});
    for (u32 v = 0; v < kMaxVars; ++v)
      if (schema[v] >= 0) vs[v] = Src{kSrcProbe, u32(schema[v])};
    s.out = head_out(vs);
    s.out_buf = -1;
    s.head_rel = r.head.rel;
    p.steps.push_back(s);
    return p;
  }

  for (u32 k = 1; k < nb; ++k) {
    const AtomR& a = r.body[order[k]];
    Step s;
    s.brel = a.rel;
    if (k == 1) s.pf = pf;
    // key candidates: constants and already-bound variables of this atom
    struct Cand { u32 col; Src src; bool is_var; };
    std::vector<Cand> cands;
    std::vector<int> newcol(kMaxVars, -1);     // first column of a variable bound here
    std::vector<Filter> wf;
    for (u32 c = 0; c < a.t.size(); ++c) {
      const Term& t = a.t[c];
      if (t.is_const) cands.push_back(Cand{c, Src{kSrcConst, t.value}, false});
      else if (schema[t.value] >= 0) cands.push_back(Cand{c, Src{kSrcProbe, u32(schema[t.value])}, true});
      else if (newcol[t.value] >= 0) wf.push_back(Filter{Src{kSrcBuild, c}, Src{kSrcBuild, u32(newcol[t.value])}, kEq});
      else newcol[t.value] = int(c);
    }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.is_var > y.is_var; });
    // Key on the bound variables; the atom's constants then select which rows
    // the index holds (t(p, 2, q) probed by p indexes only the rows whose
    // second column is 2).  Without a bound variable the constants are the key.
    size_t nvar = 0;
    while (nvar < cands.size() && cands[nvar].is_var) ++nvar;
    s.nkey = u32(std::min<size_t>(2, nvar ? nvar : cands.size()));
    u32 keycol[2] = {0, 0};
    for (u32 i = 0; i < s.nkey; ++i) { s.key[i] = cands[i].src; keycol[i] = cands[i].col; }
    // a two-column index keys on (lower column, higher column)
    if (s.nkey == 2 && keycol[0] > keycol[1]) { std::swap(keycol[0], keycol[1]); std::swap(s.key[0], s.key[1]); }
    u32 nfilt = 0, fcol[2] = {0, 0}, fval[2] = {0, 0};
    for (size_t i = s.nkey; i < cands.size(); ++i) {
      if (nvar && !cands[i].is_var && nfilt < 2) {
        fcol[nfilt] = cands[i].col;
        fval[nfilt] = cands[i].src.v;
        ++nfilt;
      } else {
        wf.push_back(Filter{Src{kSrcBuild, cands[i].col}, cands[i].src, kEq});
      }
    }
    if (nfilt == 2 && fcol[0] > fcol[1]) { std::swap(fcol[0], fcol[1]); std::swap(fval[0], fval[1]); }
    s.index = s.nkey ? get_index(a.rel, s.nkey, keycol, nfilt, fcol, fval) : kNoIndex;
    // variable sources after this join
    std::vector<Src> vs(kMaxVars, Src{kSrcConst, 0});
    std::vector<bool> have(kMaxVars, false);
    for (u32 v = 0; v < kMaxVars; ++v) {
      if (schema[v] >= 0) { vs[v] = Src{kSrcProbe, u32(schema[v])}; have[v] = true; }
      else if (newcol[v] >= 0) { vs[v] = Src{kSrcBuild, u32(newcol[v])}; have[v] = true; }
    }
    for (u32 q = 0; q < r.neq.size(); ++q) {
      if (neq_done[q]) continue;
      const u32 x = r.neq[q].first, y = r.neq[q].second;
      if (have[x] && have[y]) { wf.push_back(Filter{vs[x], vs[y], kNe}); neq_done[q] = true; }
    }
    if (wf.size() > size_t(kMaxFilters)) throw Error(FV_ENOTSUP, "too many filters on one join");
    s.wf = wf;
    if (k == nb - 1) {
      s.out = head_out(vs);
      s.out_buf = -1;
      s.head_rel = r.head.rel;
    } else {
      const std::vector<bool> need = needed_after(k, neq_done);
      std::vector<int> nschema(kMaxVars, -1);
      u32 nc = 0;
      for (u32 v = 0; v < kMaxVars; ++v) {
        if (need[v] && have[v]) {
          s.out.push_back(vs[v]);
          nschema[v] = int(nc++);
        }
      }
      if (nc == 0) {   // nothing left to carry but more atoms follow: keep one column for the row count
        for (u32 v = 0; v < kMaxVars && nc == 0; ++v)
          if (have[v]) { s.out.push_back(vs[v]); nschema[v] = int(nc++); }
      }
      if (nc > u32(kMaxCols)) throw Error(FV_ENOTSUP, "more than 6 live variables between two joins");
      Inter I;
      I.ncols = nc;
      inters_.push_back(I);
      s.out_buf = int(inters_.size() - 1);
      schema = nschema;
    }
    p.steps.push_back(s);
  }
  return p;
}

void Engine::plan_all() {
  init_plans_.clear();
  delta_plans_.clear();
  int groups = 0;
  for (u32 ri = 0; ri < rules_.size(); ++ri) {
    const RuleR& r = rules_[ri];
    init_plans_.push_back(plan_rule(ri, -1));
    for (u32 i = 0; i < r.body.size(); ++i) {
      if (!rels_[r.body[i].rel].idb) continue;
      Plan p = plan_rule(ri, int(i));
      // FV_LEARNED: a body of three or more atoms where several atoms share a
      // variable with the delta atom can start with any of them; those join
      // orders are planned too, and each round runs the one with the fewest
      // predicted intermediate rows (the default order first, so that ties
      // keep it)
      std::vector<Plan> alts;
      if (learned_ && r.body.size() >= 3) {
        for (u32 j = 0; j < r.body.size() && alts.size() < kMaxJoinOrders - 1; ++j) {
          if (j == i || j == p.second) continue;
          bool shares = false;
          for (auto& t : r.body[j].t)
            for (auto& u : r.body[i].t) shares = shares || (!t.is_const && !u.is_const && t.value == u.value);
          if (shares) alts.push_back(plan_rule(ri, int(i), int(j)));
        }
      }
      if (!alts.empty()) { p.alt = groups; p.alt_default = true; }
      delta_plans_.push_back(p);
      for (auto& q : alts) {
        q.alt = groups;
        q.active = false;
        delta_plans_.push_back(q);
      }
      if (!alts.empty()) ++groups;
    }
  }
  alt_distrusted_.assign(size_t(groups), 0);
  for (auto& r : rules_) rels_[r.head.rel].used_as_head = true;
  // Algorithm 2's difference reads an index of full on every column of a
  // derived relation (shared with any join that keys on that column alone)
  if (tune_.dedup_ranges == 1)
    for (u32 ri = 0; ri < rels_.size(); ++ri)
      if (rels_[ri].used_as_head)
        for (u32 c = 0; c < rels_[ri].arity; ++c) rels_[ri].dix[c] = get_index(ri, 1, &c, 0, nullptr, nullptr);
  // counter layout: [derived, join_out] [full_n x R] [d_begin x R]
  //   [index distinct keys] [index longest runs] [index full flags] [index rows] [HLL estimate, rows]
  //   [predicted join sizes]                                          (kept across rounds)
  //   [delta x R] [new x R] [per-join m,t] [per-intermediate count] [sketch rows]  (cleared every round)
  const int R = int(rels_.size());
  c_derived_ = 0;
  c_joinout_ = 1;
  c_full0_ = 2;
  c_dbeg0_ = c_full0_ + R;
  int next = c_dbeg0_ + R;
  c_ndv0_ = next;
  for (auto& ix : indices_) ix.c_ndv = next++;
  for (auto& ix : indices_) ix.c_maxrun = next++;
  for (auto& ix : indices_) ix.c_full = next++;
  for (auto& ix : indices_) ix.c_rows = next++;
  for (auto& ix : indices_) ix.c_top = next++;
  for (auto& Rl : rels_) Rl.c_ones = next++;
  c_hll0_ = next;
  sketches_.clear();
  if (log_joins_) {
    for (auto* plans : {&init_plans_, &delta_plans_})
      for (auto& p : *plans) {
        if (p.steps.empty() || p.steps[0].select_only || p.steps[0].nkey == 0) continue;
        Step& s0 = p.steps[0];
        if (s0.key[0].kind != kSrcProbe) continue;
        const int c1 = (s0.nkey == 2 && s0.key[1].kind == kSrcProbe) ? int(s0.key[1].v) : -1;
        const bool delta = p.delta_pos >= 0;
        auto same_filters = [&](const std::vector<Filter>& a) {
          if (a.size() != s0.pf.size()) return false;
          for (size_t f = 0; f < a.size(); ++f)
            if (a[f].op != s0.pf[f].op || a[f].a.kind != s0.pf[f].a.kind || a[f].a.v != s0.pf[f].a.v ||
                a[f].b.kind != s0.pf[f].b.kind || a[f].b.v != s0.pf[f].b.v)
              return false;
          return true;
        };
        int found = -1;
        for (size_t i = 0; i < sketches_.size(); ++i)
          if (sketches_[i].rel == p.src_rel && sketches_[i].c0 == s0.key[0].v && sketches_[i].c1 == c1 &&
              sketches_[i].delta == delta && same_filters(sketches_[i].pf))
            found = int(i);
        if (found < 0) {
          HllSketch sk;
          sk.rel = p.src_rel;
          sk.c0 = s0.key[0].v;
          sk.c1 = c1;
          sk.delta = delta;
          sk.pf = s0.pf;
          sk.ctr = next++;
          sketches_.push_back(sk);
          found = int(sketches_.size() - 1);
        }
        s0.hll = found;
      }
  }
  c_pred0_ = next;
  for (auto* plans : {&init_plans_, &delta_plans_})
    for (auto& p : *plans)
      for (auto& s : p.steps)
        if (!s.select_only) s.c_pred = next++;
  c_delta0_ = next;
  c_new0_ = c_delta0_ + R;
  c_reset_begin_ = c_delta0_;
  next = c_new0_ + R;
  for (auto* plans : {&init_plans_, &delta_plans_})
    for (auto& p : *plans)
      for (auto& s : p.steps)
        if (!s.select_only) { s.c_m = next++; s.c_t = next++; s.c_n = next++; }
  for (auto& I : inters_) I.ctr = next++;
  for (auto& ix : indices_) { ix.c_wl = next++; ix.c_moves = next++; ix.c_mrows = next++; }
  // rows passing a sketch's filters: counted afresh by every sketch launch
  for (auto& sk : sketches_) sk.ctr_rows = next++;
  n_ctr_ = next;
}

// ------------------------------------------------------------------ capacity
bool Engine::ensure_capacity(bool dry) {
  const u64 allocs_before = n_allocs_;
  // look-back status arrays and row-id scratch are sized for the largest
  // launch any round can make before capacities change again: a delta is at
  // most the previous round's new tuples, so new_cap bounds it
  u64 max_probe = 1, max_rows = 1, sort_rows = 0, word_rows = 0, moves_need = 0;
  auto plan_probe = [&](const Plan& p, bool initial) {
    const Relation& S = rels_[p.src_rel];
    const u64 n0 = initial ? S.n_full : std::max<u64>(S.n_delta, S.new_cap);
    for (size_t k = 0; k < p.steps.size(); ++k) {
      const u64 n = k == 0 ? n0 : inters_[p.steps[k - 1].out_buf].cap;
      max_probe = std::max(max_probe, n);
    }
  };
  for (auto& p : init_plans_) plan_probe(p, true);
  for (auto& p : delta_plans_) plan_probe(p, false);
  // with look-ahead a relation may take two rounds of new tuples before the
  // host sees the first
  const u64 ahead_rounds = ahead_active_ ? 2 : 1;
  // growth of the last round over the one before (>= 1; 2 without history)
  auto growth = [](u64 last, u64 prev) { return prev ? std::max(1.0, double(last) / double(prev)) : 2.0; };
  if (dry) {
    // a look-ahead round is sized before the round ahead of it is known:
    // take it only while every buffer has room for two more rounds of the
    // last round-over-round growth (and a quarter more), so that it rarely
    // overflows and runs again
    auto short_for = [&](u64 last, u64 prev, u64 cap) {
      const double g = growth(last, prev);
      return 1.25 * double(last) * g * g > double(cap);
    };
    if (deltas_.size() < 3) return true;   // no growth history yet
    for (auto& R : rels_)
      if (R.used_as_head && short_for(R.last_new, R.prev_new, R.new_cap)) return true;
    for (auto& I : inters_)
      if (short_for(I.last_used, I.prev_used, I.cap)) return true;
  }
  for (auto& R : rels_) {
    max_rows = std::max(max_rows, R.new_cap);
    if (!R.used_as_head) continue;
    const u64 need_full = R.n_full + ahead_rounds * R.new_cap;
    if (R.cap < need_full) {
      if (dry) return true;
      // doubling: each growth copies full and (with look-ahead) stops the
      // overlap of two rounds, so it should happen a logarithmic number of times
      const u64 nc = std::max<u64>(need_full, 2 * R.cap);
      for (u32 c = 0; c < R.arity; ++c) grow(R.col[c], nc * 4, R.n_full * 4);
      R.cap = nc;
    }
    // Sized for the expected size at load <= 2/3; a round that still runs out
    // of slots (bounded probing) is re-run with a larger set.  Growth is 4x
    // past the target so that the rebuild (a re-insert of all of full)
    // happens a logarithmic number of times.  Expected size: full plus the
    // new-tuple volume the buffers were sized for (new_cap anticipates 4x the
    // last round); with look-ahead also two more rounds at the last growth rate.
    u64 expect = R.n_full + std::max<u64>({3 * R.n_delta, R.new_cap / 4, R.staged, 1024});
    if (ahead_rounds == 2) {
      const double g = growth(R.last_new, R.prev_new);
      expect = std::max<u64>(expect, R.n_full + u64(1.25 * double(R.last_new) * (g + g * g)));
    }
    const u64 need_set = pow2_at_least(std::max<u64>(R.set_min, u64(double(expect) / tune_.set_load)));
    if (!tune_.dedup_ranges && (R.set_cap < R.set_min || R.set_cap < expect * 3 / 2 || R.set_stale)) {
      if (dry) return true;
      R.set_stale = false;
      release(R.set);
      R.set = alloc(need_set * (R.set32 ? 4 : 8));
      R.set_cap = need_set;
      if (R.set32) {
        launched(launch_fill_u32(R.set.as<u32>(), need_set, kEmptyKey32, stream_), "set clear");
        launched(launch_fill_u64(ctr(R.c_ones), 1, 0, stream_), "set clear");
      } else {
        launched(launch_fill_u64(R.set.as<u64>(), need_set, kEmptyKey, stream_), "set clear");
      }
      const u32* cols[3] = {R.col[0].as<u32>(), R.col[1].as<u32>(), R.col[2].as<u32>()};
      launched(launch_set_insert_rows(cols, R.arity, R.shift, R.n_full, R.set32 ? nullptr : R.set.as<u64>(),
                                      need_set - 1, stream_, R.set32 ? R.set.as<u32>() : nullptr,
                                      R.set32 ? ctr(R.c_ones) : nullptr),
               "set rebuild");
    }
    if (R.newk.bytes < R.new_cap * 8) {
      if (dry) return true;
      release(R.newk);
      release(R.newk2);
      R.newk = alloc(R.new_cap * 8);
      R.newk2 = alloc(R.new_cap * 8);
    }
    // the difference by merge: full's sorted keys and the merge's output hold
    // full after this round (its rows plus every new tuple it may append)
    const u64 need_sorted = R.n_full + std::max<u64>(R.new_cap, R.staged);
    if (merge_diff() && mdiff_cap_ < diff_sorted_scratch_words(need_sorted)) {
      if (dry) return true;
      const u64 words = diff_sorted_scratch_words(2 * need_sorted);
      release(mdiff_);
      mdiff_ = alloc(words * 8);
      mdiff_cap_ = words;
    }
    if (merge_diff() && R.sfull_cap < need_sorted) {
      if (dry) return true;
      const u64 nc = std::max<u64>(need_sorted, 2 * R.sfull_cap);
      Buf a = alloc(nc * 8), b;
      try {
        b = alloc(nc * 8);
      } catch (...) {
        release(a);
        throw;
      }
      if (R.n_full) hip(hipMemcpyAsync(a.p, R.sfull.p, R.n_full * 8, hipMemcpyDeviceToDevice, stream_), "sorted copy");
      release(R.sfull);
      release(R.sfull2);
      R.sfull = a;
      R.sfull2 = b;
      R.sfull_cap = nc;
    }
    max_rows = std::max(max_rows, R.new_cap);
  }
  for (auto& ix : indices_) {
    const Relation& R = rels_[ix.rel];
    const u64 rows = R.used_as_head ? R.n_full + R.new_cap : R.n_full;
    // The table holds distinct keys, not rows: size it from the last build's
    // count (with room to double on a derived relation), or from the rows
    // before the first build.  A build that still runs out of slots raises
    // the index's full flag and the table is rebuilt larger before the next
    // round reads it; one measured far below its table (an index over a
    // selective filter, or a low-cardinality column) gets a smaller one.
    // a derived relation's index before its first measurement also gets room
    // for the rows the first rounds may add, scaled by the share of the
    // relation's rows it keeps (all of them when the relation starts empty)
    const u64 grow_rows = !R.used_as_head ? 0
                          : R.n_full ? u64(double(ix.rows_hint) / double(R.n_full) * double(base_cap_ / 4))
                                     : base_cap_ / 4;
    u64 keys;
    if (ix.keys_seen) keys = R.used_as_head ? 2 * std::max<u64>(ix.keys_seen, 512) : ix.keys_seen;
    else if (ix.hinted && !R.used_as_head) keys = std::max<u64>(ix.keys_hint + ix.keys_hint / 4, 512);
    else if (ix.hinted)
      keys = std::max<u64>(2 * std::max<u64>(ix.keys_hint + ix.keys_hint / 4, 512), ix.keys_hint + grow_rows / 2);
    else keys = R.used_as_head ? R.n_full + std::max<u64>({3 * R.n_delta, base_cap_ / 4, 1024}) : R.n_full;
    keys = std::min<u64>(keys, rows + 1);
    u64 need = pow2_at_least(std::max<u64>(u64(double(keys) / tune_.index_load), 64));
    if (ix.grow) need = std::max<u64>(need, 4 * ix.cap);
    const bool oversized = (ix.keys_seen || ix.hinted) && ix.cap > 8 * need;
    if (ix.cap == 0 || ix.grow || double(keys) > 0.75 * double(ix.cap) || oversized) {
      if (dry) return true;
      // an intact index of a derived relation that outgrows its table moves
      // into a larger one (keys re-inserted with their runs; perm stays), a
      // build is needed otherwise
      const bool rehash = R.used_as_head && !ix.dirty && !ix.grow && ix.cap && ix.pcap.p && need > ix.cap &&
                          !tune_.index_rebuild && !use_graph_;
      Buf nt = alloc(need * sizeof(Slot)), np, nd, nw;
      try {
        if (R.used_as_head) {   // updated every round: region sizes, appended counts, work list
          np = alloc(need * 4);
          nd = alloc(need * 4);
          nw = alloc(need * 4);
        }
      } catch (...) {
        for (Buf* b : {&nt, &np, &nd}) release(*b);
        throw;
      }
      if (rehash) {
        launched(launch_index_rehash(ix.table.as<Slot>(), ix.pcap.as<u32>(), ix.cap, nt.as<Slot>(), np.as<u32>(), need,
                                     ctr(ix.c_full), stream_),
                 "index rehash");
        rehashed_.push_back(u32(&ix - &indices_[0]));
      }
      for (Buf* b : {&ix.table, &ix.pcap, &ix.dcnt, &ix.wl}) release(*b);
      ix.table = nt;
      ix.pcap = np;
      ix.dcnt = nd;
      ix.wl = nw;
      if (nd.p) launched(launch_fill_u32(ix.dcnt.as<u32>(), need, 0u, stream_), "index delta counts clear");
      ix.cap = need;
      if (!rehash) ix.dirty = true;
      ix.grow = false;
    }
    // Positions.  A loaded relation's index holds exactly its rows.  A
    // derived relation's index keeps each run in a region with room to grow
    // and moves a run that outgrows it to fresh positions (twice its size),
    // so it gets 4x the rows it may hold after this round: its measured rows
    // plus its share of the round's new tuples.  When the positions in use
    // pass half of it, it moves to an array of twice the size (the regions
    // keep their place) or, when the index must be rebuilt anyway, the build
    // packs the runs again.  An update that still runs out raises the full
    // flag and the index is rebuilt with more before the next round reads it.
    u64 want = rows;
    bool realloc_perm = ix.perm_cap < rows;
    const u64 have = ix.rows_seen ? ix.rows_seen : (ix.hinted ? ix.rows_hint : 0);
    if (!R.used_as_head && ix.hinted) {
      want = std::max<u64>(ix.rows_hint, 1);
      realloc_perm = ix.perm_cap < want;
    } else if (R.used_as_head) {
      const double share =
          ix.rows_seen && R.n_full ? std::min(1.0, double(ix.rows_seen) / double(R.n_full)) : 1.0;
      const u64 base = ix.rows_seen ? ix.rows_seen : (have ? have + grow_rows : rows);
      const u64 after = base + u64(share * double(R.new_cap));
      want = 4 * std::max<u64>(after, 4096);
      const u64 used = std::max(ix.top_seen, after);
      realloc_perm = ix.perm_cap < 2 * used || ix.perm_cap > 32 * std::max<u64>(used, 4096);
    }
    if (ix.perm_grow) {
      want = std::max<u64>(want, 2 * ix.perm_cap);
      realloc_perm = true;
    }
    want = std::min<u64>(want, u64(0xFFFFFFFFu));   // positions are 32-bit
    if (dry && (ix.perm_cap == 0 || realloc_perm)) return true;
    if (!dry) ix.perm_grow = false;
    if (!dry && (ix.perm_cap == 0 || realloc_perm)) {
      // an intact index keeps its layout: the positions in use move to the
      // new array (a streaming copy) instead of a rebuild
      const u64 used = R.used_as_head ? ix.top_seen : ix.rows_seen;
      const bool keep = !ix.dirty && ix.rows_seen && ix.perm.p && used <= want;
      Buf np = alloc(std::max<u64>(want, 1) * 4);
      if (keep && used)
        hip(hipMemcpyAsync(np.p, ix.perm.p, used * 4, hipMemcpyDeviceToDevice, stream_), "index copy");
      release(ix.perm);
      ix.perm = np;
      ix.perm_cap = want;
      if (!keep) ix.dirty = true;
    }
    if (R.used_as_head) moves_need = std::max<u64>(moves_need, ix.perm_cap / 32 + 1024);
    max_rows = std::max(max_rows, ix.cap);
    // Construction: a large build sorts (row, slot) words by slot (no
    // per-row atomics; see build_index), a small one counts by hashing.
    // The slot bits (plus one for rows outside a filter) are sorted with
    // 8-bit digits, and the row id sits above the last digit.
    u32 sort_shift = 0, sort_bits = 0;
    if (tune_.index_sort == 2 || (tune_.index_sort == 0 && rows >= (u64(1) << 20))) {
      const u32 slot_bits = bits_for(ix.cap) - 1 + (ix.nfilt ? 1 : 0);   // cap is a power of two
      const u32 shift = sort_passes(slot_bits, 8) * 8;
      const u32 row_bits = bits_for(R.cap - 1);
      if (shift + row_bits <= 64) {
        sort_shift = shift;
        sort_bits = slot_bits;
        sort_rows = std::max(sort_rows, R.cap);
      }
    }
    // An update sorts the appended rows by slot when the last round appended
    // at least 2^20 rows and the index keeps a good share of them (at least a
    // quarter of the relation's rows; the counting update skips the rows
    // outside a selective filter for free, while the sort would still pass
    // over them): mostly distinct keys then cost random table and counter
    // accesses per row, and a few hot keys serialise the counting update's
    // atomics, where the sorted words are walked in slot order.  The words fit
    // in new_cap words of scratch.  Before the first round (which reads every
    // fact as its delta) the facts stand in for the last round's rows.
    u32 upd_shift = 0;
    const double share = ix.rows_seen && R.n_full ? double(ix.rows_seen) / double(R.n_full) : 1.0;
    const u64 last_rows = deltas_.empty() ? R.n_full : R.n_delta;
    if (R.used_as_head &&
        (tune_.index_sort == 2 ||
         (tune_.index_sort == 0 && last_rows >= (u64(1) << 20) && (ix.nfilt == 0 || share >= 0.25)))) {
      const u32 slot_bits = bits_for(ix.cap) - 1 + (ix.nfilt ? 1 : 0);
      const u32 shift = sort_passes(slot_bits, 8) * 8;
      if (shift + bits_for(std::max<u64>(R.new_cap, 1) - 1) <= 64) {
        upd_shift = shift;
        sort_rows = std::max(sort_rows, R.new_cap);
      }
    }
    // (a counting update notes a word per appended row in the same scratch)
    if (R.used_as_head) word_rows = std::max(word_rows, R.new_cap);
    if (!dry) {
      ix.sort_shift = sort_shift;
      ix.sort_bits = sort_bits;
      ix.upd_shift = upd_shift;
    }
  }
  if (moves_cap_ < moves_need) {
    if (dry) return true;
    release(moves_);
    moves_ = alloc(moves_need * sizeof(RunMove));
    moves_cap_ = moves_need;
  }
  word_rows = std::max(word_rows, sort_rows);
  if (ixk_cap_ < word_rows) {
    if (dry) return true;
    release(ixk_a_); release(ixk_b_);
    ixk_a_ = alloc(word_rows * 8);
    ixk_b_ = alloc(word_rows * 8);
    ixk_cap_ = word_rows;
  }
  max_rows = std::max(max_rows, sort_rows);
  for (auto& I : inters_) {
    if (I.cap == 0) {
      if (dry) return true;
      I.cap = 1 << 16;
    }
    for (u32 c = 0; c < I.ncols; ++c)
      if (I.col[c].bytes < I.cap * 4) {
        if (dry) return true;
        release(I.col[c]);
        I.col[c] = alloc(I.cap * 4);
      }
  }
  if (m_cap_ < max_probe) {
    if (dry) return true;
    const u64 nc = std::max<u64>(max_probe, m_cap_ * 2);
    release(m_row_); release(m_start_); release(m_off_);
    m_row_ = alloc(nc * 4);
    m_start_ = alloc(nc * 4);
    m_off_ = alloc(nc * 8);
    m_cap_ = nc;
  }
  // (tiles of the smallest block size: 128 threads x 4 rows)
  const u64 tiles = (std::max(max_probe, max_rows) + 511) / 512 + 2;
  if (st_cap_ < tiles) {
    if (dry) return true;
    const u64 nc = std::max<u64>(tiles, st_cap_ * 2);
    release(st_a_); release(st_b_);
    st_a_ = alloc(nc * 8);
    st_b_ = alloc(nc * 8);
    launched(launch_fill_u64(st_a_.as<u64>(), nc, 0, stream_), "status clear");
    launched(launch_fill_u64(st_b_.as<u64>(), nc, 0, stream_), "status clear");
    st_cap_ = nc;
  }
  const u64 stiles = (max_rows + kSortTile - 1) / kSortTile + 1;
  if (st_sort_tiles_ < stiles) {
    if (dry) return true;
    const u64 nc = std::max<u64>(stiles, st_sort_tiles_ * 2);
    release(st_sort_);
    st_sort_ = alloc(nc * sort_status_words() * 8);
    launched(launch_fill_u64(st_sort_.as<u64>(), nc * sort_status_words(), 0, stream_), "status clear");
    st_sort_tiles_ = nc;
  }
  return n_allocs_ != allocs_before;
}

// ------------------------------------------------------------------ profiling
void Engine::host_time(const char* name, std::chrono::steady_clock::time_point since) {
  if (!trace_ || !trace_only_.empty()) return;
  KClass& k = kprof_[kclass(name)];
  k.launches += 1;
  k.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - since).count();
}

int Engine::kclass(const char* name) {
  for (size_t i = 0; i < kprof_.size(); ++i)
    if (kprof_[i].name == name) return int(i);
  KClass k;
  k.name = name;
  kprof_.push_back(k);
  return int(kprof_.size() - 1);
}

hipEvent_t Engine::pooled_event() {
  hipEvent_t e;
  if (!ev_pool_.empty()) { e = ev_pool_.back(); ev_pool_.pop_back(); }
  else hip(hipEventCreate(&e), "event create");
  return e;
}

// Time the launches between ev_begin and ev_end.  A single kernel (`single`)
// gets a stamp slot (the returned pointer goes into its parameters): the
// kernel stamps its own start and end on the device clock, so its time holds
// no dispatch gap.  A group of launches, or a launch being captured into a
// graph, is timed by events recorded on the stream around it.
u64* Engine::ev_begin(int cls, bool single) {
  ev_stamp_ = -1;
  ev_open_ = nullptr;
  if (!trace_) return nullptr;
  if (!trace_only_.empty() && kprof_[cls].name != trace_only_) return nullptr;
  ev_is_open_ = true;
  if (single && !capturing_ && stamps_used_ == kMaxStamps && pending_.empty()) flush_stamps();
  if (single && !capturing_ && stamps_used_ < kMaxStamps) {
    if (!stamps_dev_.p) {
      stamps_dev_ = alloc(size_t(kMaxStamps) * kStampWords * 8);
      launched(launch_fill_u64(stamps_dev_.as<u64>(), u64(kMaxStamps) * kStampWords, 0, stream_), "stamp clear");
    }
    ev_stamp_ = int(stamps_used_++);
    return stamps_dev_.as<u64>() + size_t(kStampWords) * ev_stamp_;
  }
  ev_open_ = pooled_event();
  hip(hipEventRecord(ev_open_, stream_), "event record");
  return nullptr;
}

// Drop a timing opened by ev_begin (a launch that will not be timed).
void Engine::ev_cancel() {
  if (ev_open_) ev_pool_.push_back(ev_open_);
  ev_open_ = nullptr;
  ev_is_open_ = false;
  ev_stamp_ = -1;
}

void Engine::ev_end(int cls, double bytes, int kind, int ref0, int ref1, u64 aux) {
  if (!trace_ || !ev_is_open_) return;
  ev_is_open_ = false;
  hipEvent_t e = nullptr;
  if (ev_stamp_ < 0) {
    e = pooled_event();
    hip(hipEventRecord(e, stream_), "event record");
  }
  pending_.push_back(PendingEvent{cls, ev_open_, e, bytes, kind, ref0, ref1, aux, ev_stamp_, emit_seq_});
  ev_open_ = nullptr;
  ev_stamp_ = -1;
}

// Algorithmic bytes of a launch, from the sizes read back after the round.
// kind 1 probe: aux = probe rows (or ref0 counter), ref1 = matched counter
// kind 2 write: ref0 = matched, ref1 = outputs; aux = bytes per output
// kind 3 sort pass / kind 4 hist / kind 5 dedup: ref0 = rows counter, aux = cap or arity
void Engine::collect_events(u64 upto, bool discard) {
  if (!trace_) return;
  std::vector<PendingEvent> all, later;
  for (auto& pe : pending_) (pe.seq <= upto ? all : later).push_back(pe);
  pending_.swap(later);
  if (discard) {   // launches of a look-ahead round that did nothing
    for (auto& pe : all)
      if (pe.stamp < 0) { ev_pool_.push_back(pe.a); ev_pool_.push_back(pe.b); }
    return;
  }
  const size_t n_eager = all.size();
  if (graph_replayed_) all.insert(all.end(), graph_events_.begin(), graph_events_.end());
  for (size_t idx = 0; idx < all.size(); ++idx) {
    PendingEvent& pe = all[idx];
    float ms = 0;
    if (pe.stamp >= 0) stamped_.emplace_back(pe.cls, pe.stamp);   // its time comes with flush_stamps
    else hip(hipEventElapsedTime(&ms, pe.a, pe.b), "event elapsed");
    KClass& k = kprof_[pe.cls];
    k.launches += 1;
    k.ms += ms;
    auto C = [&](int i) -> u64 { return i >= 0 ? ctr_host_[i] : 0; };
    double bytes = pe.bytes;
    u64 items = 0;
    switch (pe.kind) {
      case 1: {   // probe: key read + slot read per row, 16 B written per matched row
        const u64 rows = pe.ref0 >= 0 ? C(pe.ref0) : pe.aux;
        bytes = double(rows) * (4 + 16) + double(C(pe.ref1)) * 16;
        items = rows;
        break;
      }
      case 2: {   // write: perm + gathered build columns per output, run record per matched row
        const u64 m = C(pe.ref0), t = C(pe.ref1);
        bytes = double(t) * double(pe.aux) + double(m) * 16;
        items = t;
        break;
      }
      case 3: {   // radix pass: read + write 8 B per key
        const u64 n = std::min<u64>(C(pe.ref0), pe.aux);
        bytes = double(n) * 16;
        items = n;
        break;
      }
      case 4: {   // histogram: read 8 B per key
        const u64 n = std::min<u64>(C(pe.ref0), pe.aux);
        bytes = double(n) * 8;
        items = n;
        break;
      }
      case 7: {   // one-pass join: key + slot per probe row, row id + gathers + write per output
        const u64 rows = pe.ref0 >= 0 ? C(pe.ref0) : pe.aux;
        const u64 t = C(pe.ref1);
        bytes = double(rows) * 20 + double(t) * 16;
        items = t;
        break;
      }
      case 6: {   // fused last pass: read key, set probe, column writes of survivors
        const u64 n = C(pe.ref0), d = C(pe.ref1);
        bytes = double(n) * 16 + double(d) * 4 * double(pe.aux);
        items = n;
        break;
      }
      case 14: {   // index build: key columns read (in pe.bytes with the table), row ids written
        items = C(pe.ref0);
        bytes = pe.bytes + 4.0 * double(items);
        break;
      }
      case 15: {   // update keys: key columns read, slot found, word written per appended row
        const u64 appended = C(c_delta0_ + pe.ref0);
        bytes = double(appended) * (4.0 * double(pe.aux) + 16 + 8);
        items = appended;
        break;
      }
      case 17: case 18: case 19: {   // sorted update steps: words in slot order
        const u64 appended = C(c_delta0_ + pe.ref0);
        if (pe.kind == 17) {          // reserve: words read; slot, count, region per run head
          bytes = double(appended) * 8;
          items = appended;
        } else if (pe.kind == 18) {   // move: listed old rows read and written
          items = C(int(pe.aux & 0xFFFFFFFFu));
          bytes = double(items) * 8;
        } else {                      // fill: word read, slot and counters (in slot order), row id written
          bytes = double(appended) * (8 + 4);
          items = appended;
        }
        break;
      }
      case 10: case 11: case 12: case 13: {   // index update steps (see update_index)
        const u64 appended = C(c_delta0_ + pe.ref0), touched = C(pe.ref1);
        const double cols = double(pe.aux >> 32);
        if (pe.kind == 10) {          // count: key columns read and (slot, place) written per appended row;
          bytes = double(appended) * (4 * cols + 8) + double(touched) * 24;   // slot + counter per touched key
          items = appended;
        } else if (pe.kind == 11) {   // reserve: work list, counters, slot, region size per touched key
          bytes = double(touched) * 36;
          items = touched;
        } else if (pe.kind == 12) {   // move: listed old rows read and written
          items = C(int(pe.aux & 0xFFFFFFFFu));
          bytes = double(items) * 8;
        } else {                      // fill: (slot, place) read, row id written; slot + counter per touched key
          bytes = double(appended) * (8 + 4) + double(touched) * 20;
          items = appended;
        }
        break;
      }
      case 20: {   // difference by merge: full's and the new keys read, full's and the survivors' keys
                   // written, survivors' columns appended
        const u64 n = C(pe.ref0), d = C(pe.ref1), f = C(int(pe.aux >> 32));   // f: full after the round
        bytes = double(n) * 8 + double(f - d) * 8 + double(f) * 8 + double(d) * 4 * double(pe.aux & 0xFFFFFFFFu);
        items = n + (f - d);
        break;
      }
      case 5: {   // difference + append: key read, set probe, column writes of survivors
        const u64 n = C(pe.ref0), d = C(pe.ref1);
        bytes = double(n) * 16 + double(d) * 4 * double(pe.aux);
        items = n;
        break;
      }
      default:
        break;
    }
    k.bytes += bytes;
    k.items += items;
    if (idx < n_eager && pe.stamp < 0) {   // events owned by the graph are recorded again by the next replay
      ev_pool_.push_back(pe.a);
      ev_pool_.push_back(pe.b);
    }
  }
  graph_replayed_ = false;
}

// Times of the stamped launches so far, in one readback (the slots then start
// over).  Called when the slots run out and at the end of a run.
void Engine::flush_stamps() {
  if (!stamps_used_) return;
  std::vector<u64> w(size_t(kStampWords) * stamps_used_);
  hip(hipMemcpyAsync(w.data(), stamps_dev_.p, w.size() * 8, hipMemcpyDeviceToHost, stream_), "stamp readback");
  sync();
  for (auto& cs : stamped_) {
    const u64* s = &w[size_t(kStampWords) * cs.second];
    const u64 t0 = s[0], t1 = *std::max_element(s + 1, s + kStampWords);
    if (t0 && t1 > t0) kprof_[cs.first].ms += double(t1 - t0) / wall_khz_;   // an aborted launch stamps no end
  }
  stamped_.clear();
  launched(launch_fill_u64(stamps_dev_.as<u64>(), w.size(), 0, stream_), "stamp clear");
  stamps_used_ = 0;
}

// ------------------------------------------------------------------ execution
// The end of a read-back is awaited by polling its event (the host thread has
// nothing else to do; a blocking wait adds wake-up latency to every round).
void Engine::wait_event(hipEvent_t e) {
  for (;;) {
    const hipError_t q = hipEventQuery(e);
    if (q == hipSuccess) return;
    if (q != hipErrorNotReady) hip(q, "round wait");
  }
}

void Engine::read_counters() {
  ctr_host_ = rb_host_[0];
  flags_host_ = reinterpret_cast<u32*>(ctr_host_ + n_ctr_);
  hip(hipMemcpyAsync(ctr_host_, ctr_dev_.p, size_t(n_ctr_) * 8 + kFlagBytes, hipMemcpyDeviceToHost, stream_),
      "counter readback");
  hip(hipEventRecord(rb_ev_[0], stream_), "event record");
  wait_event(rb_ev_[0]);
  collect_events(emit_seq_, false);
  if (flags_host_[1]) {
    terminal = true;
    throw Error(FV_EINVAL, "internal: join scratch too small");
  }
}

void Engine::exec_plan(Plan& p) {
  u32* flags = flags_dev_.as<u32>();
  u32* ticket = ticket_dev_.as<u32>();
  const bool initial = p.delta_pos < 0;
  for (size_t k = 0; k < p.steps.size(); ++k) {
    Step& s = p.steps[k];
    const u32* pcol[kMaxCols] = {};
    RowRange src{};
    u64 probe_bound;
    if (k == 0) {
      const Relation& S = rels_[p.src_rel];
      for (u32 c = 0; c < S.arity; ++c) pcol[c] = S.col[c].as<u32>();
      const u32 ri = u32(&S - &rels_[0]);
      src.begin_ctr = initial ? nullptr : ctr(c_dbeg0_ + int(ri));
      src.end_ctr = ctr(c_full0_ + int(ri));
      src.cap = S.cap ? S.cap : S.n_full;
      probe_bound = initial ? S.n_full : std::max<u64>(S.n_delta, S.new_cap);
    } else {
      const Inter& I = inters_[p.steps[k - 1].out_buf];
      for (u32 c = 0; c < I.ncols; ++c) pcol[c] = I.col[c].as<u32>();
      src.end_ctr = ctr(I.ctr);
      src.cap = I.cap;
      probe_bound = I.cap;
    }
    OutSpec o{};
    o.ncols = u32(s.out.size());
    for (u32 c = 0; c < o.ncols; ++c) o.src[c] = s.out[c];
    if (s.out_buf >= 0) {
      Inter& I = inters_[s.out_buf];
      for (u32 c = 0; c < I.ncols; ++c) o.cols[c] = I.col[c].as<u32>();
      o.count = ctr(I.ctr);
      o.cap = I.cap;
    } else {
      Relation& H = rels_[s.head_rel];
      o.packed = 1;
      for (u32 c = 0; c < H.arity; ++c) o.shift[c] = H.shift[c];
      o.keys = H.newk.as<u64>();
      o.count = ctr(c_new0_ + int(s.head_rel));
      o.cap = H.new_cap;
      if (H.hist_by_writers) {
        o.hist = hist_dev_.as<u32>() + size_t(s.head_rel) * kHistWords;
        o.hist_passes = sort_passes(H.bits, 8);
      }
    }
    if (s.select_only) {
      SelectParams sp{};
      for (int c = 0; c < kMaxCols; ++c) sp.pcol[c] = pcol[c];
      sp.src = src;
      sp.n_filter = u32(s.pf.size());
      for (u32 f = 0; f < sp.n_filter; ++f) sp.filt[f] = s.pf[f];
      sp.out = o;
      sp.join_out_stat = ctr(c_joinout_);
      sp.abort = flags + kFlagVoid;
      sp.overflow = flags;
      const int kc = kclass("select");
      sp.ts = ev_begin(kc, true);
      launched(launch_select(sp, std::max<u64>(probe_bound, 1), stream_, block_for(0, probe_bound)), "select launch");
      ev_end(kc, 0, 0);
      continue;
    }
    const Relation& B = rels_[s.brel];
    if (s.fused) {
      // presized output: probe and write in one pass
      FusedJoinParams fp{};
      for (int c = 0; c < kMaxCols; ++c) fp.pcol[c] = pcol[c];
      fp.src = src;
      fp.n_pf = u32(s.pf.size());
      for (u32 f = 0; f < fp.n_pf; ++f) fp.pf[f] = s.pf[f];
      fp.nkey = s.nkey;
      fp.key[0] = s.key[0];
      fp.key[1] = s.key[1];
      const Index* fx = s.index != kNoIndex ? &indices_[s.index] : nullptr;
      if (fx) {
        fp.table = fx->table.as<Slot>();
        fp.mask = fx->cap - 1;
        fp.perm = fx->perm.as<u32>();
      } else {
        fp.build_rows_ctr = ctr(c_full0_ + int(s.brel));
        fp.build_cap = B.cap ? B.cap : B.n_full;
      }
      for (u32 c = 0; c < B.arity; ++c) fp.bcol[c] = B.col[c].as<u32>();
      fp.n_filter = u32(s.wf.size());
      for (u32 f = 0; f < fp.n_filter; ++f) fp.filt[f] = s.wf[f];
      fp.out = o;
      fp.out_t = ctr(s.c_t);
      fp.out_n = ctr(s.c_n);
      fp.join_out_stat = ctr(c_joinout_);
      fp.abort = flags + kFlagVoid;
      fp.overflow = flags;
      const int kf = kclass("join_onepass");
      fp.ts = ev_begin(kf, true);
      launched(launch_join_fused(fp, std::max<u64>(probe_bound, 1), stream_, block_for(0, probe_bound)),
               "one-pass join launch");
      ev_end(kf, 0, 7, s.c_n, s.c_t, probe_bound);
      continue;
    }
    ProbeParams pp{};
    for (int c = 0; c < kMaxCols; ++c) pp.pcol[c] = pcol[c];
    pp.src = src;
    pp.n_pf = u32(s.pf.size());
    for (u32 f = 0; f < pp.n_pf; ++f) pp.pf[f] = s.pf[f];
    pp.nkey = s.nkey;
    pp.key[0] = s.key[0];
    pp.key[1] = s.key[1];
    const Index* ix = s.index != kNoIndex ? &indices_[s.index] : nullptr;
    if (ix) {
      pp.table = ix->table.as<Slot>();
      pp.mask = ix->cap - 1;
    } else {
      pp.build_rows_ctr = ctr(c_full0_ + int(s.brel));
      pp.build_cap = B.cap ? B.cap : B.n_full;
    }
    pp.m_row = m_row_.as<u32>();
    pp.m_start = m_start_.as<u32>();
    pp.m_off = m_off_.as<u64>();
    pp.m_cap = m_cap_;
    pp.out_m = ctr(s.c_m);
    pp.out_t = ctr(s.c_t);
    pp.out_n = ctr(s.c_n);
    pp.st_m = st_a_.as<u64>();
    pp.st_t = st_b_.as<u64>();
    pp.ticket = ticket;
    pp.epoch_base = epoch_base();
    pp.epoch_off = next_epoch();
    pp.abort = flags + kFlagVoid;
    pp.fatal = flags + kFlagFatal;
    const int kp = kclass("join_probe");
    pp.ts = ev_begin(kp, true);
    launched(launch_probe(pp, std::max<u64>(probe_bound, 1), 0, stream_, block_for(0, probe_bound)), "probe launch");
    ev_end(kp, 0, 1, s.c_n, s.c_m, probe_bound);

    WriteParams wp{};
    for (int c = 0; c < kMaxCols; ++c) wp.pcol[c] = pcol[c];
    for (u32 c = 0; c < B.arity; ++c) wp.bcol[c] = B.col[c].as<u32>();
    wp.perm = ix ? ix->perm.as<u32>() : nullptr;
    wp.m_row = m_row_.as<u32>();
    wp.m_start = m_start_.as<u32>();
    wp.m_off = m_off_.as<u64>();
    wp.m_cap = m_cap_;
    wp.in_m = ctr(s.c_m);
    wp.in_t = ctr(s.c_t);
    wp.n_filter = u32(s.wf.size());
    for (u32 f = 0; f < wp.n_filter; ++f) wp.filt[f] = s.wf[f];
    wp.out = o;
    wp.join_out_stat = ctr(c_joinout_);
    wp.abort = flags + kFlagFatal;   // the probe ran out of scratch: write nothing
    wp.abort2 = flags + kFlagVoid;
    wp.overflow = flags;
    u32 nbuild = 0;
    for (auto& sc : s.out) nbuild += sc.kind == kSrcBuild ? 1 : 0;
    for (auto& f : s.wf) nbuild += (f.a.kind == kSrcBuild) + (f.b.kind == kSrcBuild);
    const u64 out_bytes = o.packed ? 8 : 4ull * o.ncols;
    const int kw = kclass("join_write");
    wp.ts = ev_begin(kw, true);
    launched(launch_write(wp, std::max<u64>(o.cap, 1), stream_, block_for(0, probe_bound)), "write launch");
    ev_end(kw, 0, 2, s.c_m, s.c_t, (ix ? 4 : 0) + 4ull * nbuild + out_bytes);
  }
}

// sort the relation's new keys, take the difference against full, append
void Engine::finish_relation(Relation& R, bool in_round) {
  const int ri = int(&R - &rels_[0]);
  u32* flags = flags_dev_.as<u32>();
  SortParams sp{};
  sp.a = R.newk.as<u64>();
  sp.b = R.newk2.as<u64>();
  sp.n_ctr = ctr(c_new0_ + ri);
  sp.cap = R.new_cap;
  sp.n_hint = R.last_new;
  sp.bits = R.bits;
  sp.digit_bits = tune_.radix_bits;
  sp.max_blocks = tune_.max_blocks;
  sp.hist = hist_dev_.as<u32>() + size_t(ri) * kHistWords;
  sp.status = st_sort_.as<u64>();
  sp.ticket = ticket_dev_.as<u32>();
  sp.epoch_base = epoch_base();
  sp.abort = flags;
  const u32 passes = sort_passes(R.bits, tune_.radix_bits);
  // the last radix pass can take the difference itself when there is a set
  const bool fuse = tune_.fuse_dedup && R.idb && passes > 0 && !tune_.dedup_ranges;
  if (!(in_round && R.hist_by_writers)) {   // else the writers counted the digits
    const int kh = kclass("sort_hist");
    ev_begin(kh);
    launched(launch_rs_hist(sp, stream_, !in_round), "hist launch");
    ev_end(kh, 0, 4, c_new0_ + ri, -1, R.new_cap);
  }
  u64* src = sp.a;
  u64* dst = sp.b;
  const int kpass = kclass("sort_pass");
  const int kfused = kclass("sort_pass_dedup");
  SortFuse fz{};
  if (fuse) {
    fz.set = R.set32 ? nullptr : R.set.as<u64>();
    fz.set32 = R.set32 ? R.set.as<u32>() : nullptr;
    fz.ones = R.set32 ? ctr(R.c_ones) : nullptr;
    fz.set_mask = R.set_cap - 1;
    fz.set_full = flags + 2;
    for (u32 c = 0; c < R.arity; ++c) {
      fz.cols[c] = R.col[c].as<u32>();
      fz.shift[c] = R.shift[c];
      fz.width[c] = R.width[c];
    }
    fz.full_n = ctr(c_full0_ + ri);
    fz.out_delta = ctr(c_delta0_ + ri);
    fz.arity = R.arity;
  }
  for (u32 pass = 0; pass < passes; ++pass) {
    const bool last_fused = fuse && pass + 1 == passes;
    sp.ts = ev_begin(last_fused ? kfused : kpass, true);
    launched(launch_rs_pass(sp, pass, src, dst, next_epoch(), stream_, last_fused ? &fz : nullptr),
             "sort pass launch");
    ev_end(last_fused ? kfused : kpass, 0, last_fused ? 6 : 3, c_new0_ + ri, c_delta0_ + ri,
           last_fused ? R.arity : R.new_cap);
    std::swap(src, dst);
  }
  if (fuse) return;
  DedupParams dp{};
  dp.keys = src;
  dp.src.end_ctr = ctr(c_new0_ + ri);
  dp.src.cap = R.new_cap;
  const bool use_set = R.idb && !tune_.dedup_ranges;
  dp.set = use_set && !R.set32 ? R.set.as<u64>() : nullptr;
  dp.set32 = use_set && R.set32 ? R.set.as<u32>() : nullptr;
  dp.ones = use_set && R.set32 ? ctr(R.c_ones) : nullptr;
  if (merge_diff() && R.used_as_head) {
    // the difference against full's sorted keys, which it merges with the
    // new keys into the second copy (taken over when the round succeeds)
    dp.sorted_full = R.sfull.as<u64>();
    dp.merged = R.sfull2.as<u64>();
    dp.mtile = mdiff_.as<u64>();
    R.merged_this_round = true;
  }
  if (tune_.dedup_ranges == 1 && in_round && R.used_as_head) {
    // full is empty before the first round (ingest), so only rounds need the test
    dp.rd.ncol = R.arity;
    for (u32 c = 0; c < R.arity; ++c) {
      const Index& ix = indices_[R.dix[c]];
      dp.rd.table[c] = ix.table.as<Slot>();
      dp.rd.mask[c] = ix.cap - 1;
      dp.rd.perm[c] = ix.perm.as<u32>();
      dp.rd.fcol[c] = R.col[c].as<u32>();
    }
  }
  dp.set_mask = R.set_cap ? R.set_cap - 1 : 0;
  dp.set_full = flags + 2;
  for (u32 c = 0; c < R.arity; ++c) {
    dp.cols[c] = R.col[c].as<u32>();
    dp.shift[c] = R.shift[c];
    dp.width[c] = R.width[c];
  }
  dp.full_n = ctr(c_full0_ + ri);
  dp.arity = R.arity;
  dp.out_delta = ctr(c_delta0_ + ri);
  dp.status = st_a_.as<u64>();
  dp.ticket = ticket_dev_.as<u32>();
  dp.epoch_base = epoch_base();
  dp.epoch_off = next_epoch();
  dp.abort = flags;
  const int kd = kclass("dedup_append");
  dp.ts = ev_begin(kd, true);
  if (dp.sorted_full) {
    launched(launch_diff_sorted(dp, R.n_full + std::max<u64>(R.new_cap, 1), stream_, block_for(1, R.new_cap)),
             "difference launch");
    ev_end(kd, 0, 20, c_new0_ + ri, c_delta0_ + ri, (u64(c_full0_ + ri) << 32) | R.arity);
  } else {
    launched(launch_dedup(dp, std::max<u64>(R.new_cap, 1), stream_, block_for(1, R.new_cap)), "dedup launch");
    ev_end(kd, 0, 5, c_new0_ + ri, c_delta0_ + ri, R.arity);
  }
}

// A round that succeeded (or the ingest) merged the survivors into the second
// sorted copy of full: it becomes the current one.
void Engine::take_merged_full() {
  for (auto& R : rels_) {
    if (!R.merged_this_round) continue;
    std::swap(R.sfull, R.sfull2);
    R.merged_this_round = false;
    graph_dirty_ = true;   // a captured round holds the old pointers
  }
}

void Engine::commit_relation(Relation& R) {
  const int ri = int(&R - &rels_[0]);
  u32* flags = flags_dev_.as<u32>();
  CommitParams cp{};
  cp.full_n = ctr(c_full0_ + ri);
  cp.d_begin = ctr(c_dbeg0_ + ri);
  cp.delta = ctr(c_delta0_ + ri);
  cp.new_count = nullptr;
  cp.derived = ctr(c_derived_);
  cp.abort = flags;
  cp.abort2 = flags + 2;
  launched(launch_commit(cp, stream_), "commit launch");
}

void Engine::build_index(Index& ix) {
  const Relation& R = rels_[ix.rel];
  IndexParams p{};
  for (u32 c = 0; c < R.arity; ++c) p.col[c] = R.col[c].as<u32>();
  p.src.end_ctr = ctr(c_full0_ + int(ix.rel));
  p.src.cap = R.cap;
  p.nkey = ix.nkey;
  p.keycol[0] = ix.keycol[0];
  p.keycol[1] = ix.keycol[1];
  p.nfilt = ix.nfilt;
  for (u32 f = 0; f < 2; ++f) { p.fcol[f] = ix.fcol[f]; p.fval[f] = ix.fval[f]; }
  p.table = ix.table.as<Slot>();
  p.cap = ix.cap;
  p.perm = ix.perm.as<u32>();
  p.perm_cap = ix.perm_cap;
  p.status = st_a_.as<u64>();
  p.ticket = ticket_dev_.as<u32>();
  p.epoch_base = epoch_base();
  p.epoch_off = next_epoch();
  p.abort = flags_dev_.as<u32>();
  p.ndv = ix.c_ndv >= 0 ? ctr(ix.c_ndv) : nullptr;
  p.maxrun = ix.c_maxrun >= 0 ? ctr(ix.c_maxrun) : nullptr;
  p.full = ix.c_full >= 0 ? ctr(ix.c_full) : nullptr;
  p.rows = ix.c_rows >= 0 ? ctr(ix.c_rows) : nullptr;
  if (R.used_as_head) {   // regions with room to grow, bump pointer past the last
    p.pcap = ix.pcap.as<u32>();
    p.top = ctr(ix.c_top);
    p.wl = ix.wl.as<u32>();   // the sorted build notes each run's first word here
  }
  const int kc = kclass("index_build");
  ev_begin(kc);
  if (ix.sort_shift) {
    // sorted build: (row, slot) words, a radix sort over the slot bits, runs
    // (the keys kernel counts the sort's digits: no histogram pass)
    u32* ihist = hist_dev_.as<u32>() + rels_.size() * kHistWords;
    launched(launch_index_slotkeys(p, R.cap, ixk_a_.as<u64>(), ix.sort_shift, ihist, sort_passes(ix.sort_bits, 8),
                                   stream_),
             "index keys launch");
    SortParams sp{};
    sp.a = ixk_a_.as<u64>();
    sp.b = ixk_b_.as<u64>();
    sp.n_ctr = p.src.end_ctr;
    sp.cap = R.cap;
    sp.bits = ix.sort_bits;
    sp.digit_bits = 8;
    sp.max_blocks = tune_.max_blocks;
    sp.hist = hist_dev_.as<u32>() + rels_.size() * kHistWords;
    sp.status = st_sort_.as<u64>();
    sp.ticket = ticket_dev_.as<u32>();
    sp.epoch_base = epoch_base();
    sp.abort = flags_dev_.as<u32>();
    if (sort_passes(ix.sort_bits, 8) > 8) launched(launch_rs_hist(sp, stream_, true), "index hist launch");
    u64* src = sp.a;
    u64* dst = sp.b;
    for (u32 pass = 0; pass < sort_passes(ix.sort_bits, 8); ++pass) {
      launched(launch_rs_pass(sp, pass, src, dst, next_epoch(), stream_), "index sort pass launch");
      std::swap(src, dst);
    }
    launched(launch_index_runs(p, R.cap, src, ix.sort_shift, stream_), "index runs launch");
  } else {
    launched(launch_index_build(p, std::max<u64>(R.cap, 1), stream_), "index launch");
  }
  // algorithmic bytes: every row's key (and filter) columns read once, each
  // indexed row id written once, the table cleared and scanned
  ev_end(kc, double(R.n_full) * 4.0 * (ix.nkey + ix.nfilt) + double(ix.cap) * 32.0, 14, ix.c_rows);
  ix.dirty = false;
}

// Bring the join indices of derived relations up to date with the rows the
// round appended (launch_index_update): only the keys that got rows are
// touched.  Used for intact indices in eager rounds; a captured round
// rebuilds them instead (a replayed graph cannot know which keys it touches).
void Engine::update_index(Index& ix) {
  const Relation& R = rels_[ix.rel];
  IndexParams p{};
  for (u32 c = 0; c < R.arity; ++c) p.col[c] = R.col[c].as<u32>();
  p.src.begin_ctr = ctr(c_dbeg0_ + int(ix.rel));
  p.src.end_ctr = ctr(c_full0_ + int(ix.rel));
  p.src.cap = R.cap;
  p.nkey = ix.nkey;
  p.keycol[0] = ix.keycol[0];
  p.keycol[1] = ix.keycol[1];
  p.nfilt = ix.nfilt;
  for (u32 f = 0; f < 2; ++f) { p.fcol[f] = ix.fcol[f]; p.fval[f] = ix.fval[f]; }
  p.table = ix.table.as<Slot>();
  p.cap = ix.cap;
  p.perm = ix.perm.as<u32>();
  p.perm_cap = ix.perm_cap;
  p.abort = flags_dev_.as<u32>();
  p.abort2 = flags_dev_.as<u32>() + kFlagSetFull;
  p.ndv = ctr(ix.c_ndv);
  p.maxrun = ctr(ix.c_maxrun);
  p.full = ctr(ix.c_full);
  p.rows = ctr(ix.c_rows);
  p.pcap = ix.pcap.as<u32>();
  p.top = ctr(ix.c_top);
  p.dcnt = ix.dcnt.as<u32>();
  p.wl = ix.wl.as<u32>();
  p.wl_n = ctr(ix.c_wl);
  p.moves = moves_.as<RunMove>();
  p.moves_n = ctr(ix.c_moves);
  p.moves_cap = moves_cap_;
  p.moved_rows = ctr(ix.c_mrows);
  const u64 dcap = std::max<u64>(R.new_cap, 1);
  // each step is its own kernel class, timed by its own stamps (a step that
  // gets no stamp slot goes untimed)
  auto stamps = [&](const char* const* names, int count, int kind0, u64* ts) {
    for (int k = 0; k < count; ++k) {
      const int cls = kclass(names[k]);
      ts[k] = reinterpret_cast<u64>(ev_begin(cls, true));
      if (ts[k]) ev_end(cls, 0, kind0 + k, int(ix.rel), ix.c_wl, (u64(ix.nkey + ix.nfilt) << 32) | u64(ix.c_mrows));
      else ev_cancel();
    }
  };
  u64 tsv[4];
  u64* ts[4];
  if (!ix.upd_shift) {
    const char* names[4] = {"index_upd_count", "index_upd_reserve", "index_upd_move", "index_upd_fill"};
    stamps(names, 4, 10, tsv);
    for (int k = 0; k < 4; ++k) ts[k] = reinterpret_cast<u64*>(tsv[k]);
    p.rword = ixk_a_.as<u64>();   // new_cap words (sized in ensure_capacity)
    launched(launch_index_update(p, dcap, ix.cap, ts, stream_), "index update launch");
    return;
  }
  // many appended rows with short runs: sort the appended rows by slot first
  SortParams sp{};
  sp.a = ixk_a_.as<u64>();
  sp.b = ixk_b_.as<u64>();
  sp.n_ctr = ctr(c_delta0_ + int(ix.rel));   // rows appended by the commit
  sp.cap = dcap;
  sp.bits = bits_for(ix.cap) - 1 + (ix.nfilt ? 1 : 0);
  sp.digit_bits = 8;
  sp.max_blocks = tune_.max_blocks;
  sp.hist = hist_dev_.as<u32>() + rels_.size() * kHistWords;
  sp.status = st_sort_.as<u64>();
  sp.ticket = ticket_dev_.as<u32>();
  sp.epoch_base = epoch_base();
  sp.abort = flags_dev_.as<u32>();
  {
    // the keys kernel counts the sort's digits as it writes the words
    const int kc = kclass("index_upd_keys");
    ev_begin(kc);
    launched(launch_index_update_keys(p, dcap, ixk_a_.as<u64>(), ix.upd_shift, sp.hist, sort_passes(sp.bits, 8),
                                      stream_),
             "index keys launch");
    ev_end(kc, 0, 15, int(ix.rel), -1, u64(ix.nkey + ix.nfilt));
  }
  if (sort_passes(sp.bits, 8) > 8) {
    const int kh = kclass("sort_hist");
    ev_begin(kh);
    launched(launch_rs_hist(sp, stream_, true), "index hist launch");
    ev_end(kh, 0, 4, c_delta0_ + int(ix.rel), -1, dcap);
  }
  u64* src = sp.a;
  u64* dst = sp.b;
  const int kpass = kclass("sort_pass");
  for (u32 pass = 0; pass < sort_passes(sp.bits, 8); ++pass) {
    sp.ts = ev_begin(kpass, true);
    launched(launch_rs_pass(sp, pass, src, dst, next_epoch(), stream_), "index sort pass launch");
    ev_end(kpass, 0, 3, c_delta0_ + int(ix.rel), -1, dcap);
    std::swap(src, dst);
  }
  const char* names[3] = {"index_upds_reserve", "index_upd_move", "index_upds_fill"};
  stamps(names, 3, 17, tsv);
  for (int k = 0; k < 3; ++k) ts[k] = reinterpret_cast<u64*>(tsv[k]);
  launched(launch_index_update_sorted(p, dcap, src, ix.upd_shift, ts, stream_), "index update launch");
}

void Engine::build_indices(bool idb_only) {
  for (auto& ix : indices_) {
    if (idb_only && !rels_[ix.rel].used_as_head) continue;
    if (idb_only && !tune_.index_rebuild && !use_graph_ && !capturing_ && !ix.dirty && ix.pcap.p) update_index(ix);
    else build_index(ix);
  }
}

// Load the staged facts of every relation: pack, radix-sort, drop repeats,
// and for relations that are also derived, seed the tuple set.
void Engine::ingest() {
  u64 total = 0;
  for (auto& R : rels_) total += R.staged;
  const u64 base_cap = small_caps_ ? 256 : pow2_at_least(std::max<u64>(1 << 16, 2 * total));
  base_cap_ = base_cap;
  for (auto& R : rels_) {
    R.new_cap = std::max<u64>(R.staged, R.used_as_head ? base_cap : 1);
    if (!R.used_as_head) {   // read-only relation: exactly its facts
      R.cap = std::max<u64>(R.staged, 1);
      for (u32 c = 0; c < R.arity; ++c) R.col[c] = alloc(R.cap * 4);
      R.newk = alloc(R.new_cap * 8);
      R.newk2 = alloc(R.new_cap * 8);
    }
  }
  for (auto& I : inters_) I.cap = base_cap;
  ensure_capacity();
  hip(hipMemsetAsync(ctr_dev_.p, 0, size_t(n_ctr_) * 8, stream_), "counter clear");
  hip(hipMemsetAsync(flags_dev_.p, 0, kFlagBytes, stream_), "flag clear");
  phases_ = 0;
  begin_phase();
  for (auto& R : rels_) {
    if (!R.staged) continue;
    const int ri = int(&R - &rels_[0]);
    const u32* cols[3] = {R.stage[0].as<u32>(), R.stage[1].as<u32>(), R.stage[2].as<u32>()};
    launched(launch_pack(cols, R.arity, R.shift, R.staged, R.newk.as<u64>(), stream_), "pack launch");
    launched(launch_fill_u64(ctr(c_new0_ + ri), 1, R.staged, stream_), "fill");
    finish_relation(R, false);
  }
  for (auto& R : rels_)
    if (R.staged) commit_relation(R);
  read_counters();
  take_merged_full();
  for (auto& R : rels_) {
    const int ri = int(&R - &rels_[0]);
    R.n_full = ctr_host_[c_full0_ + ri];
    R.d_begin = ctr_host_[c_dbeg0_ + ri];
    R.seeds = R.n_full;
    R.n_delta = 0;
    for (int c = 0; c < 3; ++c) release(R.stage[c]);
    R.staged = 0;
    if (!R.used_as_head) { release(R.newk); release(R.newk2); R.new_cap = 0; }
    else R.new_cap = base_cap;
  }
  // after ingest the delta of every relation is empty; round 0 reads full
  hip(hipMemsetAsync(ctr_dev_.p, 0, 8, stream_), "derived clear");
}

// Enqueue one round: prologue (counters, overflow flag, histograms, epoch
// base), the joins of every plan, sort + difference + merge per derived
// relation, and the rebuild of indices on derived relations.  `all_plans`
// keeps plans whose delta is empty (a captured round must not depend on
// host-side sizes).
void Engine::emit_round(bool initial, bool all_plans, bool sticky) {
  launched(launch_round_prologue(ctr(c_reset_begin_), u64(n_ctr_ - c_reset_begin_), flags_dev_.as<u32>(),
                                 hist_dev_.as<u32>(), hist_dev_.bytes / 4, epoch_base(), stream_, sticky),
           "round prologue");
  epoch_off_ = 1;
  // the writers of a relation's new keys count the sort's 8-bit digits as
  // they write (no histogram pass), unless a one-pass join writes some of them
  for (auto& R : rels_) R.hist_by_writers = R.used_as_head && tune_.radix_bits == 8;
  for (auto* plans : {&init_plans_, &delta_plans_})
    for (auto& p : *plans)
      for (auto& s : p.steps)
        if (p.active && s.out_buf < 0 && s.fused) rels_[s.head_rel].hist_by_writers = false;
  if (initial) {
    for (auto& p : init_plans_) exec_plan(p);
  } else {
    for (auto& p : delta_plans_)
      if (p.active && (all_plans || rels_[p.src_rel].n_delta > 0)) exec_plan(p);
  }
  // test hook: this emission fails as if a join had overflowed (before any
  // sort, difference or commit), so the round runs again
  if (!capturing_) {
    ++emitted_;
    if (fail_rounds_.count(emitted_))
      launched(launch_fill_u32(flags_dev_.as<u32>() + kFlagOverflow, 1, 1u, stream_), "test failure");
  }
  // every relation's difference first, then the commits: a round that runs
  // out of set space commits nothing
  for (auto& R : rels_)
    if (R.used_as_head) finish_relation(R, true);
  for (auto& R : rels_)
    if (R.used_as_head) commit_relation(R);
  build_indices(true);
  if (log_joins_) emit_sketches_and_prediction(false);
}

void Engine::drop_graph() {
  if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
  if (graph_) (void)hipGraphDestroy(graph_);
  graph_exec_ = nullptr;
  graph_ = nullptr;
  for (auto& pe : graph_events_) { ev_pool_.push_back(pe.a); ev_pool_.push_back(pe.b); }
  graph_events_.clear();
}

// Capture one recursive round into a graph.  With tracing, the per-kernel
// events are captured too; if the runtime refuses that, capture without them.
bool Engine::capture_round() {
  drop_graph();
  for (int attempt = 0; attempt < 2; ++attempt) {
    const bool with_events = trace_ && graph_events_ok_;
    const bool saved_trace = trace_;
    if (!with_events) trace_ = false;
    pending_.clear();
    bool ok = hipStreamBeginCapture(stream_, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      capturing_ = true;
      try {
        emit_round(false, true);
      } catch (const Error&) {
        ok = false;
      }
      capturing_ = false;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(stream_, &g);
      ok = ok && e == hipSuccess && g;
      if (ok) {
        ok = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0) == hipSuccess;
        graph_ = g;
        if (!ok) { (void)hipGraphDestroy(g); graph_ = nullptr; graph_exec_ = nullptr; }
      } else if (g) {
        (void)hipGraphDestroy(g);
      }
    }
    trace_ = saved_trace;
    (void)hipGetLastError();
    if (ok) {
      graph_events_.swap(pending_);
      pending_.clear();
      graph_dirty_ = false;
      graph_fused_steps_ = fused_steps_;
      ++graph_captures_;
      return true;
    }
    for (auto& pe : pending_) { ev_pool_.push_back(pe.a); ev_pool_.push_back(pe.b); }
    pending_.clear();
    if (!with_events) break;
    graph_events_ok_ = false;
  }
  return false;
}

// A presized one-pass join hands each wave the outputs of its own probe
// rows, so it stays balanced only while no key owns many build rows; a join
// whose build index has a long run (measured by the index's last build) runs
// as count-then-write, which spreads outputs evenly over the grid.
constexpr u64 kOnePassMaxRun = 256;

void Engine::choose_join_algorithms(bool initial) {
  fused_steps_.clear();
  for (auto& p : initial ? init_plans_ : delta_plans_) {
    fused_steps_.push_back(p.active);
    for (auto& s : p.steps) {
      s.fused = p.active && use_fused_ && !s.select_only && s.index != kNoIndex &&
                ctr_host_[indices_[s.index].c_maxrun] <= kOnePassMaxRun;
      fused_steps_.push_back(s.fused);
    }
  }
}

// FV_LEARNED: of each group of plans that differ in join order, run the one
// whose intermediate results (every join output but the last, whose size
// the order does not change) the predictor expects to be smallest, if that
// is under half of what it expects from the default order and if even the
// worst case of that order (probe rows times each build index's longest run)
// stays within four times that expectation: a prediction that is far too low
// on skewed keys then cannot pick an order that explodes.  The predictions
// are those made at the end of the previous round.  A group whose chosen
// order once overflowed its presized buffers keeps the default order.
void Engine::choose_join_orders() {
  for (size_t i = 0; i < delta_plans_.size();) {
    if (delta_plans_[i].alt < 0) { ++i; continue; }
    const int g = delta_plans_[i].alt;
    size_t j = i;
    std::vector<double> rows, worst;
    double default_rows = 0;
    for (; j < delta_plans_.size() && delta_plans_[j].alt == g; ++j) {
      const Plan& p = delta_plans_[j];
      const Relation& S = rels_[p.src_rel];
      double r = 0, w = 0;
      double bound = double(p.steps.empty() || p.steps[0].hll < 0 ? S.n_delta
                                                                   : ctr_host_[sketches_[p.steps[0].hll].ctr_rows]);
      for (size_t k = 0; k + 1 < p.steps.size(); ++k) {
        const Step& st = p.steps[k];
        if (st.c_pred >= 0) r += double(ctr_host_[st.c_pred]);
        bound *= st.index != kNoIndex ? double(std::max<u64>(ctr_host_[indices_[st.index].c_maxrun], 1))
                                      : double(ctr_host_[c_full0_ + int(st.brel)]);
        w += bound;
      }
      rows.push_back(r);
      worst.push_back(w);
      if (p.alt_default) default_rows = r;
    }
    size_t best = j;   // j: keep the default
    if (!alt_distrusted_[size_t(g)])
      for (size_t k = i; k < j; ++k)
        if (!delta_plans_[k].alt_default && 2.0 * rows[k - i] < default_rows &&
            worst[k - i] <= 4.0 * default_rows && (best == j || rows[k - i] < rows[best - i]))
          best = k;
    for (size_t k = i; k < j; ++k) delta_plans_[k].active = best == j ? delta_plans_[k].alt_default : k == best;
    if (best != j) ++reordered_rounds_;
    i = j;
  }
}

void Engine::run_round(bool initial) {
  auto th = std::chrono::steady_clock::now();
  start_ctr_.assign(ctr_host_, ctr_host_ + n_ctr_);
  use_fused_ = learned_;
  if (learned_ && !initial) choose_join_orders();
  if (learned_) size_from_predictions(initial);
  choose_join_algorithms(initial);
  for (;;) {
    if (ensure_capacity()) graph_dirty_ = true;
    if (phases_ + 2 >= (kEpochMask + 1) / kEpochStride - 96) graph_dirty_ = true;
    bool any_dirty = !rehashed_.empty();
    for (auto& ix : indices_) any_dirty = any_dirty || ix.dirty;
    if (any_dirty) {
      // an index whose storage grew holds nothing yet: rebuild it over the
      // current full relation before any join reads it (and check that the
      // indices moved to larger tables kept every key)
      begin_phase();
      std::vector<u32> built;
      built.swap(rehashed_);
      for (u32 i = 0; i < indices_.size(); ++i)
        if (indices_[i].dirty) {
          build_index(indices_[i]);
          built.push_back(i);
        }
      verify_builds(built);
    }
    if (phases_ + 2 >= (kEpochMask + 1) / kEpochStride - 96) begin_phase();   // clears status arrays
    host_time("host_prepare", th);   // sizing, growth, index rebuilds: the GPU waits
    bool replayed = false;
    if (graph_exec_ && graph_fused_steps_ != fused_steps_) graph_dirty_ = true;
    if (!initial && use_graph_) {
      if (graph_dirty_ || !graph_exec_) {
        if (!capture_round()) use_graph_ = false;
      }
      if (use_graph_) {
        hip(hipGraphLaunch(graph_exec_, stream_), "graph launch");
        replayed = true;
        ++graph_replays_;
      }
    }
    th = std::chrono::steady_clock::now();
    if (!replayed) emit_round(initial, false);
    host_time("host_enqueue", th);
    ++phases_;
    graph_replayed_ = replayed;
    th = std::chrono::steady_clock::now();
    read_counters();
    host_time("host_wait", th);
    th = std::chrono::steady_clock::now();
    if (!flags_host_[0] && !flags_host_[2]) break;
    grow_after_failure(initial);
  }
  finish_round(initial, th);
}

// A round raised a flag: it committed nothing.  Grow what was short (or fall
// back to exact joins) before the round runs again.
void Engine::grow_after_failure(bool initial) {
  ++redo_;
  bool any_fused = false;
  for (bool f : fused_steps_) any_fused = any_fused || f;
  if (any_fused && flags_host_[0]) {
    // a presized one-pass join ran out of room: run the round again with
    // exact count-then-write joins, and in the default join order where the
    // predictions had picked another (its intermediates can be far larger
    // than predicted; it is not tried again in this fixpoint)
    ++overflows_;
    use_fused_ = false;
    if (!initial)
      for (auto& p : delta_plans_)
        if (p.alt >= 0) {
          if (p.active && !p.alt_default) alt_distrusted_[size_t(p.alt)] = 1;
          p.active = p.alt_default;
        }
    choose_join_algorithms(initial);
    graph_dirty_ = true;
  }
  if (flags_host_[2]) {
    // a tuple set ran out of slots: the round committed nothing, but its
    // difference passes may have inserted keys; rebuild every set, larger
    for (auto& R : rels_)
      if (R.used_as_head) { R.set_min = 2 * std::max<u64>(R.set_cap, 1); R.set_stale = true; }
    graph_dirty_ = true;
  }
  // a buffer overflowed: grow whatever was short and run the round again
  for (auto& R : rels_) {
    if (!R.used_as_head) continue;
    const u64 need = ctr_host_[c_new0_ + int(&R - &rels_[0])];
    if (need > R.new_cap) R.new_cap = pow2_at_least(std::max<u64>(need + need / 4, R.new_cap * 2));
  }
  // (only the intermediates of the plans the rerun runs)
  for (auto& p : initial ? init_plans_ : delta_plans_) {
    if (!p.active) continue;
    for (auto& st : p.steps) {
      if (st.out_buf < 0) continue;
      Inter& I = inters_[size_t(st.out_buf)];
      const u64 need = ctr_host_[I.ctr];
      if (need > I.cap) I.cap = pow2_at_least(std::max<u64>(need + need / 4, I.cap * 2));
    }
  }
}

// A round that raised no flag: size the next one from it and take over its
// counters (full, delta, derived) on the host.
void Engine::finish_round(bool initial, std::chrono::steady_clock::time_point th) {
  take_merged_full();
  if (log_joins_) log_joins(initial);
  // (a program without recursive rules derives nothing after round 0)
  if (!learned_ && !delta_plans_.empty()) {
    // size the next round from this one: outputs tend to grow round over
    // round, and a buffer that overflows costs a whole re-run of the round
    // (4x while small, 2x past 2^24 rows, where memory rather than a re-run
    // is the scarcer resource)
    // (twice that with look-ahead, whose rounds are sized a round earlier)
    const u64 f = ahead_active_ ? 2 : 1;
    auto ahead = [f](u64 used) { return f * (used < (u64(1) << 24) ? 4 * used : 2 * used); };
    for (auto& R : rels_) {
      if (!R.used_as_head) continue;
      const u64 want = ahead(ctr_host_[c_new0_ + int(&R - &rels_[0])]);
      if (want > R.new_cap) R.new_cap = pow2_at_least(want);
    }
    for (auto& I : inters_) {
      const u64 want = ahead(ctr_host_[I.ctr]);
      if (want > I.cap) I.cap = pow2_at_least(want);
    }
  }
  for (auto& R : rels_)
    if (R.used_as_head) {
      R.prev_new = R.last_new;
      R.last_new = ctr_host_[c_new0_ + int(&R - &rels_[0])];
    }
  for (auto& I : inters_) {
    I.prev_used = I.last_used;
    I.last_used = ctr_host_[I.ctr];
  }
  note_index_builds();
  u64 total = 0;
  for (auto& R : rels_) {
    const int ri = int(&R - &rels_[0]);
    if (!R.used_as_head) { R.n_delta = 0; continue; }
    R.n_full = ctr_host_[c_full0_ + ri];
    R.d_begin = ctr_host_[c_dbeg0_ + ri];
    R.n_delta = R.n_full - R.d_begin;
    total += R.n_delta;
  }
  join_out_ = ctr_host_[c_joinout_];
  deltas_.push_back(total);
  host_time("host_finish", th);
}

// Rounds with one round of look-ahead.  The next round is enqueued before
// this one's counters are back on the host, so that the host's read-back,
// sizing and launches overlap the GPU's work instead of separating rounds.
// Every kernel takes its sizes from device counters and every buffer was
// sized for two rounds ahead (the look-ahead is only taken when nothing has
// to grow), so the early round computes what it would have computed later.
// It runs all delta plans (an empty delta costs a launch that finds nothing),
// and its prologue is sticky: if the round before it raises a flag, the
// look-ahead round does nothing, and both are discarded and re-run as usual.
// A round after the fixpoint (empty delta) finds nothing and is dropped.
// Applies to eager plain rounds whose joins read no index of a derived
// relation (those indices are updated between rounds on the host's word).
bool Engine::can_look_ahead() const {
  // (the difference by merge swaps full's sorted copy after each round the host has seen succeed)
  if (tune_.lookahead || learned_ || log_joins_ || use_graph_ || delta_plans_.empty() || merge_diff()) return false;
  for (auto& ix : indices_)
    if (rels_[ix.rel].used_as_head) return false;
  return true;
}

void Engine::run_with_look_ahead() {
  using clk = std::chrono::steady_clock;
  constexpr u64 kPhaseLimit = (kEpochMask + 1) / kEpochStride - 96;
  if (!rb_host_[1]) {
    hip(hipHostMalloc(reinterpret_cast<void**>(&rb_host_[1]), size_t(n_ctr_) * 8 + kFlagBytes, hipHostMallocDefault),
        "pinned alloc");
    hip(hipEventCreateWithFlags(&rb_ev_[1], hipEventDisableTiming), "event create");
  }
  choose_join_algorithms(false);
  ahead_active_ = true;   // buffers are sized for two rounds from here on
  int slot = 0;
  auto emit = [&](bool sticky, u64& seq) {
    const int s = slot;
    slot ^= 1;
    seq = ++emit_seq_;
    emit_round(false, true, sticky);
    ++phases_;
    hip(hipMemcpyAsync(rb_host_[s], ctr_dev_.p, size_t(n_ctr_) * 8 + kFlagBytes, hipMemcpyDeviceToHost, stream_),
        "counter readback");
    hip(hipEventRecord(rb_ev_[s], stream_), "event record");
    return s;
  };
  auto drop = [&](int s, u64 seq) {   // a look-ahead round that did nothing
    wait_event(rb_ev_[s]);
    collect_events(seq, true);
  };
  int cur = -1, nxt = -1;
  u64 cur_seq = 0, nxt_seq = 0;
  for (;;) {
    auto th = clk::now();
    if (cur < 0) {
      ensure_capacity();
      if (phases_ + 2 >= kPhaseLimit) begin_phase();   // clears status arrays
      host_time("host_prepare", th);
      th = clk::now();
      cur = emit(false, cur_seq);
      host_time("host_enqueue", th);
    }
    if (nxt < 0 && phases_ + 3 < kPhaseLimit && !ensure_capacity(true)) {
      th = clk::now();
      nxt = emit(true, nxt_seq);
      host_time("host_enqueue", th);
    }
    th = clk::now();
    wait_event(rb_ev_[cur]);
    ctr_host_ = rb_host_[cur];
    flags_host_ = reinterpret_cast<u32*>(ctr_host_ + n_ctr_);
    collect_events(cur_seq, false);
    host_time("host_wait", th);
    if (flags_host_[1]) {
      terminal = true;
      throw Error(FV_EINVAL, "internal: join scratch too small");
    }
    th = clk::now();
    if (flags_host_[0] || flags_host_[2]) {
      if (nxt >= 0) drop(nxt, nxt_seq);
      nxt = -1;
      grow_after_failure(false);
      cur = -1;
      continue;
    }
    finish_round(false, th);
    if (deltas_.back() == 0) {
      if (nxt >= 0) drop(nxt, nxt_seq);
      break;
    }
    cur = nxt;
    cur_seq = nxt_seq;
    nxt = -1;
  }
}

// Before an index's first build: one sketch launch per batch of indices (the
// index's key columns under its row filter) estimates the distinct keys and
// counts the rows the index will hold, so that tables and row arrays start at
// their size instead of the relation's (an index over a selective filter or a
// low-cardinality column holds far fewer keys than its relation has rows).
void Engine::presize_indices() {
  std::vector<u32> todo;
  for (u32 i = 0; i < indices_.size(); ++i) {
    const Index& ix = indices_[i];
    const Relation& R = rels_[ix.rel];
    // a small loaded relation is sized from its rows: a table a few times
    // too large costs less than the sketch launch and its read-back
    if (!R.used_as_head && R.n_full < (u64(1) << 18)) continue;
    if (!ix.keys_seen && !ix.hinted) todo.push_back(i);
  }
  if (todo.empty()) return;
  Buf regs = alloc(size_t(kHllBatch) * kHllRegs * 4);
  Buf out;
  try {
    out = alloc(todo.size() * 16);
  } catch (...) {
    release(regs);
    throw;
  }
  launched(launch_fill_u32(regs.as<u32>(), u64(kHllBatch) * kHllRegs, 0u, stream_), "sketch clear");
  launched(launch_fill_u64(out.as<u64>(), 2 * todo.size(), 0, stream_), "sketch clear");
  for (size_t b0 = 0; b0 < todo.size(); b0 += kHllBatch) {
    HllBatch batch{};
    u64 rows_hint = 1;
    for (size_t k = b0; k < todo.size() && batch.n < kHllBatch; ++k) {
      const Index& ix = indices_[todo[k]];
      const Relation& R = rels_[ix.rel];
      HllParams& hp = batch.s[batch.n];
      for (u32 c = 0; c < R.arity; ++c) hp.col[c] = R.col[c].as<u32>();
      hp.c0 = ix.keycol[0];
      hp.c1 = ix.nkey == 2 ? int(ix.keycol[1]) : -1;
      hp.src.end_ctr = ctr(c_full0_ + int(ix.rel));
      hp.src.cap = std::max<u64>(R.cap, 1);
      hp.n_pf = ix.nfilt;
      for (u32 f = 0; f < ix.nfilt; ++f)
        hp.pf[f] = Filter{Src{kSrcProbe, ix.fcol[f]}, Src{kSrcConst, ix.fval[f]}, kEq};
      hp.regs = regs.as<u32>() + size_t(batch.n) * kHllRegs;
      hp.estimate = out.as<u64>() + 2 * k;
      hp.rows = out.as<u64>() + 2 * k + 1;
      rows_hint = std::max<u64>(rows_hint, R.n_full);
      ++batch.n;
    }
    launched(launch_hll_batch(batch, rows_hint, stream_), "index sketch");
  }
  std::vector<u64> h(2 * todo.size());
  hip(hipMemcpyAsync(h.data(), out.p, h.size() * 8, hipMemcpyDeviceToHost, stream_), "sketch readback");
  sync();
  for (size_t k = 0; k < todo.size(); ++k) {
    Index& ix = indices_[todo[k]];
    double est;
    std::memcpy(&est, &h[2 * k], 8);
    ix.keys_hint = std::min<u64>(u64(est > 0 ? est : 0) + 1, std::max<u64>(h[2 * k + 1], 1));
    ix.rows_hint = h[2 * k + 1];
    ix.hinted = true;
  }
  release(regs);
  release(out);
}

// Builds that a round's joins are about to read must be complete: read their
// flags back and rebuild any that ran out of slots or positions, larger,
// until none does.  Their counts then size the next round.
void Engine::verify_builds(std::vector<u32> built) {
  for (int attempt = 0; attempt < 24 && !built.empty(); ++attempt) {
    std::vector<u64> c(n_ctr_);
    hip(hipMemcpyAsync(c.data(), ctr_dev_.p, size_t(n_ctr_) * 8, hipMemcpyDeviceToHost, stream_), "build check");
    sync();
    bool again = false;
    for (u32 i : built) {
      Index& ix = indices_[i];
      const u64 full = c[ix.c_full];
      if (full) {
        if (full & 1) ix.grow = true;
        if (full & 2) ix.perm_grow = true;
        ix.keys_seen = ix.rows_seen = 0;
        ix.hinted = false;   // outgrown its sketch: size from the relation instead
        ix.dirty = true;
        again = true;
      } else if (c[ix.c_rows]) {   // an empty index says nothing about its size to come
        ix.keys_seen = std::max<u64>(c[ix.c_ndv], 1);
        ix.rows_seen = c[ix.c_rows];
      }
      ix.top_seen = c[ix.c_top];
    }
    if (!again) return;
    ensure_capacity();
    begin_phase();
    built.clear();
    built.swap(rehashed_);
    for (u32 i = 0; i < indices_.size(); ++i)
      if (indices_[i].dirty) {
        build_index(indices_[i]);
        built.push_back(i);
      }
  }
  if (!built.empty()) throw Error(FV_ENOMEM, "a join index did not fit after repeated growth");
}

// After a round: the distinct-key counts of the indices just built size their
// tables for the next round; an index whose build ran out of slots is
// incomplete and is rebuilt larger before any join reads it.
void Engine::note_index_builds() {
  for (auto& ix : indices_) {
    ix.top_seen = ctr_host_[ix.c_top];
    const u64 full = ctr_host_[ix.c_full];
    if (full) {
      if (full & 1) ix.grow = true;
      if (full & 2) ix.perm_grow = true;
      ix.dirty = true;   // incomplete: rebuilt before any join reads it
      // its counts cover only what fitted: size the rebuild from the
      // relation's rows instead, so that it cannot fall short as well
      ix.rows_seen = 0;
      ix.keys_seen = 0;
      ix.hinted = false;
      continue;
    }
    if (!ctr_host_[ix.c_rows]) continue;   // empty: keep sizing from the relation
    ix.rows_seen = ctr_host_[ix.c_rows];
    ix.keys_seen = std::max<u64>(ctr_host_[ix.c_ndv], 1);
  }
}

// ------------------------------------------------------------------ learned predictor
void Engine::setup_learning() {
  for (auto& sk : sketches_) {   // zero here; each estimate clears them again after use
    sk.regs = alloc(kHllRegs * 4);
    launched(launch_fill_u32(sk.regs.as<u32>(), kHllRegs, 0u, stream_), "sketch clear");
  }
  if (!learned_) return;
  predictor_dev_ = alloc(kMlpParams * 4);
  hip(hipMemcpyAsync(predictor_dev_.p, predictor_.data(), kMlpParams * 4, hipMemcpyHostToDevice, stream_),
      "predictor copy");
  auto build = [&](std::vector<Plan>& plans, std::vector<PredSpec>& out, Buf& dev) {
    out.clear();
    for (auto& p : plans) {
      u32 k = 0;
      for (auto& st : p.steps) {
        if (st.select_only) continue;
        PredSpec sp{};
        sp.probe_full = c_full0_ + int(p.src_rel);
        sp.probe_dbeg = p.delta_pos >= 0 ? c_dbeg0_ + int(p.src_rel) : -1;
        sp.build_full = c_full0_ + int(st.brel);
        sp.ndv_build = st.index != kNoIndex ? indices_[st.index].c_ndv : -1;
        sp.maxrun_build = st.index != kNoIndex ? indices_[st.index].c_maxrun : -1;
        sp.rows_build = st.index != kNoIndex ? indices_[st.index].c_rows : -1;
        sp.probe_rows = (k == 0 && st.hll >= 0) ? sketches_[st.hll].ctr_rows : -1;
        sp.hll = (k == 0 && st.hll >= 0) ? sketches_[st.hll].ctr : -1;
        sp.nkey = st.nkey;
        sp.nfilt = u32(st.wf.size());
        sp.step = k++;
        sp.out = st.c_pred;
        out.push_back(sp);
      }
    }
    if (!out.empty()) {
      dev = alloc(out.size() * sizeof(PredSpec));
      hip(hipMemcpyAsync(dev.p, out.data(), out.size() * sizeof(PredSpec), hipMemcpyHostToDevice, stream_),
          "spec copy");
    }
  };
  build(init_plans_, pspec_init_, pspec_init_dev_);
  build(delta_plans_, pspec_delta_, pspec_delta_dev_);
  sync();   // the host vectors above are released/reused after this call
}

// HLL sketches of the probe keys the next round's first joins will use, then
// (FV_LEARNED) the predictor over every join of that round.
void Engine::emit_sketches_and_prediction(bool initial) {
  HllBatch batch{};
  u64 rows_hint = 1;
  auto flush = [&]() {
    if (!batch.n) return;
    const int kc = kclass("hll_sketch");
    ev_begin(kc);
    launched(launch_hll_batch(batch, rows_hint, stream_), "hll");
    ev_end(kc, 0, 0);
    batch.n = 0;
    rows_hint = 1;
  };
  for (auto& sk : sketches_) {
    if (sk.delta == initial) continue;
    const Relation& R = rels_[sk.rel];
    RowRange rr{};
    rr.begin_ctr = sk.delta ? ctr(c_dbeg0_ + int(sk.rel)) : nullptr;
    rr.end_ctr = ctr(c_full0_ + int(sk.rel));
    rr.cap = std::max<u64>(R.cap, 1);
    HllParams hp{};
    for (u32 c = 0; c < R.arity; ++c) hp.col[c] = R.col[c].as<u32>();
    hp.c0 = sk.c0;
    hp.c1 = sk.c1;
    hp.src = rr;
    hp.n_pf = u32(sk.pf.size());
    for (u32 f = 0; f < hp.n_pf; ++f) hp.pf[f] = sk.pf[f];
    hp.regs = sk.regs.as<u32>();
    hp.estimate = ctr(sk.ctr);
    hp.rows = ctr(sk.ctr_rows);
    batch.s[batch.n++] = hp;
    rows_hint = std::max<u64>(rows_hint, sk.delta ? R.n_full + R.new_cap : R.n_full);
    if (batch.n == kHllBatch) flush();
  }
  flush();
  if (!learned_) return;
  const std::vector<PredSpec>& v = initial ? pspec_init_ : pspec_delta_;
  const Buf& d = initial ? pspec_init_dev_ : pspec_delta_dev_;
  if (v.empty()) return;
  const int kc = kclass("predict");
  ev_begin(kc);
  launched(launch_predict(d.as<PredSpec>(), u32(v.size()), ctr_dev_.as<u64>(), predictor_dev_.as<float>(), stream_),
           "predict");
  ev_end(kc, 0, 0);
}

// FV_LEARNED: grow the round's output buffers to 1.25x the predicted sizes.
void Engine::size_from_predictions(bool initial) {
  std::vector<u64> need_new(rels_.size(), 0);
  for (auto& p : initial ? init_plans_ : delta_plans_) {
    const Relation& S = rels_[p.src_rel];
    if (!p.active || (!initial && S.n_delta == 0)) continue;
    double probe = 0;   // rows entering the current step (estimated past the first)
    for (size_t k = 0; k < p.steps.size(); ++k) {
      const Step& st = p.steps[k];
      u64 want;
      if (k == 0)
        probe = double(st.hll >= 0 ? ctr_host_[sketches_[st.hll].ctr_rows] : (initial ? S.n_full : S.n_delta));
      if (st.select_only) {
        want = initial ? S.n_full : S.n_delta;
      } else {
        // presize to 2x the larger of the prediction and the uniform-key
        // estimate (probe rows x the build index's mean run), within
        // [1024, 2^27] rows: a short buffer costs a re-run of the round, a
        // long one only memory; a join larger than that is served by the
        // overflow fallback's exact count
        double uniform = probe;
        if (st.index != kNoIndex) {
          const Index& ix = indices_[st.index];
          const double keys = double(std::max<u64>(ctr_host_[ix.c_ndv], 1));
          uniform = probe * std::max(1.0, double(ctr_host_[ix.c_rows]) / keys);
        }
        const double est = std::max(double(ctr_host_[st.c_pred]), uniform);
        want = u64(std::min(2.0 * est + 1024.0, double(u64(1) << 27)));
        probe = est;
      }
      if (st.out_buf >= 0) {
        Inter& I = inters_[st.out_buf];
        if (I.cap < want) I.cap = pow2_at_least(want);
      } else {
        need_new[st.head_rel] += want;
      }
    }
  }
  // a relation's new-tuple buffer (and the tuple set and indices sized from
  // it) is presized to at most 2^28 rows; more comes from the exact fallback
  for (size_t r = 0; r < rels_.size(); ++r) {
    const u64 want = std::min<u64>(need_new[r], u64(1) << 28);
    if (rels_[r].used_as_head && rels_[r].new_cap < want) rels_[r].new_cap = pow2_at_least(want);
  }
}

// One trace row per join executed in the round just finished: the features as
// they stood when the round started, the true output size, the prediction.
void Engine::log_joins(bool initial) {
  auto S0 = [&](int i) -> double { return i >= 0 ? double(start_ctr_[i]) : 0.0; };
  for (auto& p : initial ? init_plans_ : delta_plans_) {
    const Relation& S = rels_[p.src_rel];
    const u64 n_src = initial ? S.n_full : S.n_delta;   // mirrors still hold the round's start
    if (!p.active || (!initial && n_src == 0)) continue;
    u32 k = 0;
    for (size_t i = 0; i < p.steps.size(); ++i) {
      const Step& st = p.steps[i];
      if (st.select_only) continue;
      double probe;
      double ndv_p;
      if (k == 0) {
        probe = st.hll >= 0 ? S0(sketches_[st.hll].ctr_rows) : double(n_src);
        ndv_p = probe;
        if (st.hll >= 0) {
          double e;
          const u64 bits = start_ctr_[sketches_[st.hll].ctr];
          std::memcpy(&e, &bits, 8);
          if (e < ndv_p) ndv_p = e;
        }
      } else {
        probe = double(std::min<u64>(ctr_host_[inters_[p.steps[i - 1].out_buf].ctr],
                                     inters_[p.steps[i - 1].out_buf].cap));
        ndv_p = probe;
      }
      const double build = st.index != kNoIndex ? S0(indices_[st.index].c_rows) : S0(c_full0_ + int(st.brel));
      const double ndv_b = st.index != kNoIndex ? S0(indices_[st.index].c_ndv) : 1.0;
      float f[kTraceCols];
      join_features(probe, build, ndv_b, ndv_p, st.nkey, u32(st.wf.size()), k, f);
      const double m = double(ctr_host_[st.c_t]);
      f[8] = float(std::log2(1.0 + m) / 16.0);
      f[9] = -1.f;
      if (learned_) {
        const double pr = S0(st.c_pred);
        f[9] = float(pr);
        qerrors_.push_back(std::max((m + 1) / (pr + 1), (pr + 1) / (m + 1)));
      }
      trace_rows_.insert(trace_rows_.end(), f, f + kTraceCols);
      ++k;
    }
  }
}

void Engine::alloc_control() {
  if (n_ctr_ < 8) n_ctr_ = 8;
  // the counters and the four flag words are one buffer (and one pinned
  // host copy), so that a round's read-back is a single copy
  ctr_dev_ = alloc(size_t(n_ctr_) * 8 + kFlagBytes);
  flags_dev_.p = static_cast<char*>(ctr_dev_.p) + size_t(n_ctr_) * 8;
  flags_dev_.bytes = kFlagBytes;
  ticket_dev_ = alloc(16);
  // one histogram region per relation, and one for sorted index builds
  hist_dev_ = alloc((rels_.size() + 1) * kHistWords * 4);
  hip(hipMemsetAsync(ticket_dev_.p, 0, 16, stream_), "ticket clear");
  hip(hipMemsetAsync(flags_dev_.p, 0, kFlagBytes, stream_), "flag clear");
  hip(hipHostMalloc(reinterpret_cast<void**>(&rb_host_[0]), size_t(n_ctr_) * 8 + kFlagBytes, hipHostMallocDefault),
      "pinned alloc");
  ctr_host_ = rb_host_[0];
  flags_host_ = reinterpret_cast<u32*>(ctr_host_ + n_ctr_);
  hip(hipEventCreateWithFlags(&rb_ev_[0], hipEventDisableTiming), "event create");
}

void Engine::run(fv_stats* stats) {
  if (ran_) throw Error(FV_ESTATE, "the fixpoint already ran on this context");
  if (terminal) throw Error(FV_ESTATE, "context is in an error state");
  ran_ = true;
  if (host_mode_) { run_host(stats); return; }
  const auto t0 = std::chrono::steady_clock::now();
  fit_packing();
  plan_all();
  alloc_control();
  setup_learning();
  ingest();
  presize_indices();
  ensure_capacity();
  begin_phase();
  build_indices(false);
  {
    std::vector<u32> all(indices_.size());
    for (u32 i = 0; i < all.size(); ++i) all[i] = i;
    verify_builds(all);
  }
  if (log_joins_) {
    emit_sketches_and_prediction(true);
    read_counters();
  }
  deltas_.clear();
  run_round(true);
  if (deltas_.back() != 0) {
    if (can_look_ahead()) run_with_look_ahead();
    else while (deltas_.back() != 0) run_round(false);
  }
  const auto t1 = std::chrono::steady_clock::now();
  flush_stamps();
  if (stats) {
    stats->iterations = u32(deltas_.size());
    stats->redo_rounds = redo_;
    u64 derived = 0;
    for (auto& R : rels_)
      if (R.used_as_head) derived += R.n_full - R.seeds;
    stats->derived_tuples = derived;
    stats->join_output_tuples = join_out_;
    stats->ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats->graph_captures = graph_captures_;
    stats->graph_replays = graph_replays_;
    stats->overflows = overflows_;
    stats->predicted_joins = u32(qerrors_.size());
    stats->reordered_rounds = reordered_rounds_;
    stats->qerror_median = 0;
    stats->qerror_max = 0;
    if (!qerrors_.empty()) {
      std::vector<double> q = qerrors_;
      std::sort(q.begin(), q.end());
      stats->qerror_median = q[q.size() / 2];
      stats->qerror_max = q.back();
    }
  }
}

// ------------------------------------------------------------------ export
void Engine::export_rel(u32 rel, u32* const* cols, u64 capacity, u64* n_out, bool on_device) {
  if (rel >= rels_.size()) throw Error(FV_EINVAL, "bad relation handle");
  if (!ran_) throw Error(FV_ESTATE, "export is allowed after the fixpoint ran");
  Relation& R = rels_[rel];
  const u64 n = R.n_full;
  if (n_out) *n_out = n;
  if (!cols) return;
  if (capacity < n) throw Error(FV_ETRUNC, "export capacity too small");
  if (n == 0) return;
  for (u32 c = 0; c < R.arity; ++c)
    if (!cols[c]) throw Error(FV_EINVAL, "null output column");
  if (host_mode_) { host_export(rel, cols, n, on_device); return; }
  if (batch_) {   // this instance's run of the batch result, shifted back to its own ids
    Engine& M = *batch_->merged;
    const u64 b = batch_->bounds[rel][inst_];
    const u32 back = u32(0u - u32(u64(inst_) * batch_->stride));
    for (u32 c = 0; c < R.arity; ++c) {
      Buf t = M.alloc(n * 4);
      try {
        M.hip(hipMemcpyAsync(t.p, batch_->cols[rel][c].as<u32>() + b, n * 4, hipMemcpyDeviceToDevice, M.stream_),
              "slice copy");
        M.launched(launch_add_u32(t.as<u32>(), n, back, M.stream_), "relabel back");
        M.hip(hipMemcpyAsync(cols[c], t.p, n * 4, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             M.stream_), "export copy");
        M.sync();
      } catch (...) {
        M.release(t);
        throw;
      }
      M.release(t);
    }
    return;
  }
  // shifts already give lexicographic (col0, col1, col2) order: pack, sort, unpack
  Buf a, b;
  Buf tmp[3];
  try {
    a = alloc(n * 8);
    b = alloc(n * 8);
    const u32* in[3] = {R.col[0].as<u32>(), R.col[1].as<u32>(), R.col[2].as<u32>()};
    launched(launch_pack(in, R.arity, R.shift, n, a.as<u64>(), stream_), "pack launch");
    const u64 stiles = (n + kSortTile - 1) / kSortTile + 1;
    if (st_sort_tiles_ < stiles) {
      release(st_sort_);
      st_sort_ = alloc(stiles * sort_status_words() * 8);
      launched(launch_fill_u64(st_sort_.as<u64>(), stiles * sort_status_words(), 0, stream_), "status clear");
      st_sort_tiles_ = stiles;
    }
    SortParams sp{};
    sp.a = a.as<u64>();
    sp.b = b.as<u64>();
    sp.n_const = n;
    sp.cap = n;
    sp.bits = R.bits;
    sp.hist = hist_dev_.as<u32>();
    sp.digit_bits = tune_.radix_bits;
    sp.max_blocks = tune_.max_blocks;
    sp.status = st_sort_.as<u64>();
    sp.ticket = ticket_dev_.as<u32>();
    sp.epoch_base = epoch_base();
    sp.abort = nullptr;
    begin_phase();
    launched(launch_rs_hist(sp, stream_), "hist launch");
    u64* s = sp.a;
    u64* d = sp.b;
    for (u32 pass = 0; pass < sort_passes(R.bits, tune_.radix_bits); ++pass) {
      launched(launch_rs_pass(sp, pass, s, d, next_epoch(), stream_), "sort pass launch");
      std::swap(s, d);
    }
    u32* outc[3] = {nullptr, nullptr, nullptr};
    for (u32 c = 0; c < R.arity; ++c) {
      if (on_device) outc[c] = cols[c];
      else { tmp[c] = alloc(n * 4); outc[c] = tmp[c].as<u32>(); }
    }
    launched(launch_unpack(s, n, R.arity, R.shift, R.width, outc, stream_), "unpack launch");
    if (compacted_) map_back(outc, R.arity, n, true);
    if (!on_device)
      for (u32 c = 0; c < R.arity; ++c)
        hip(hipMemcpyAsync(cols[c], outc[c], n * 4, hipMemcpyDeviceToHost, stream_), "export copy");
    sync();
  } catch (...) {
    release(a); release(b);
    for (auto& t : tmp) release(t);
    throw;
  }
  release(a); release(b);
  for (auto& t : tmp) release(t);
}

}  // namespace fv

namespace fv {

// ------------------------------------------------------------------ batched form
// Many independent instances of one program, each over its own facts, are
// evaluated as a single fixpoint: instance k's values are shifted into the
// id range [k * stride, (k + 1) * stride).  When no rule has constants and
// every rule body is connected through shared variables, a derived tuple
// only combines values of one instance, so the union's fixpoint restricted
// to instance k's range is instance k's fixpoint.  Every operator then runs
// as one launch over all instances, and an instance whose delta is empty
// simply contributes no rows.
BatchResult::~BatchResult() {
  if (!merged) return;
  if (merged->touched_device_) (void)hipStreamSynchronize(merged->stream_);
  for (auto& rc : cols)
    for (auto& b : rc) merged->release(b);
}

void Engine::run_batch(Engine* const* es, u32 n, fv_stats* stats) {
  if (n == 0 || !es || !es[0]) throw Error(FV_EINVAL, "empty batch");
  Engine& E0 = *es[0];
  for (u32 k = 0; k < n; ++k) {
    const Engine& E = *es[k];
    if (!es[k]) throw Error(FV_EINVAL, "null context in batch");
    if (E.ran_ || E.terminal) throw Error(FV_ESTATE, "every batched context must be fresh");
    if (E.host_mode_) throw Error(FV_ENOTSUP, "the batched form runs on the GPU only");
    if (E.rels_.size() != E0.rels_.size() || E.rules_.size() != E0.rules_.size())
      throw Error(FV_EINVAL, "batched contexts must hold the same program");
    for (size_t r = 0; r < E.rels_.size(); ++r)
      if (E.rels_[r].name != E0.rels_[r].name || E.rels_[r].arity != E0.rels_[r].arity)
        throw Error(FV_EINVAL, "batched contexts must declare the same relations in the same order");
    for (size_t i = 0; i < E.rules_.size(); ++i) {
      const RuleR &a = E.rules_[i], &b = E0.rules_[i];
      auto same_atom = [](const AtomR& x, const AtomR& y) {
        if (x.rel != y.rel || x.t.size() != y.t.size()) return false;
        for (size_t c = 0; c < x.t.size(); ++c)
          if (x.t[c].value != y.t[c].value || x.t[c].is_const != y.t[c].is_const) return false;
        return true;
      };
      bool same = same_atom(a.head, b.head) && a.body.size() == b.body.size() && a.neq == b.neq;
      for (size_t j = 0; same && j < a.body.size(); ++j) same = same_atom(a.body[j], b.body[j]);
      if (!same) throw Error(FV_EINVAL, "batched contexts must hold the same rules");
    }
  }
  for (const RuleR& r : E0.rules_) {
    for (const AtomR* a : {&r.head}) for (auto& t : a->t) if (t.is_const) throw Error(FV_ENOTSUP, "batched rules may not use constants");
    for (auto& a : r.body) for (auto& t : a.t) if (t.is_const) throw Error(FV_ENOTSUP, "batched rules may not use constants");
    // body connectivity through shared variables
    const size_t nb = r.body.size();
    std::vector<bool> in(nb, false);
    std::vector<bool> var(kMaxVars, false);
    in[0] = true;
    for (auto& t : r.body[0].t) var[t.value] = true;
    for (bool grew = true; grew;) {
      grew = false;
      for (size_t j = 0; j < nb; ++j) {
        if (in[j]) continue;
        bool touch = false;
        for (auto& t : r.body[j].t) touch = touch || var[t.value];
        if (touch) { in[j] = true; grew = true; for (auto& t : r.body[j].t) var[t.value] = true; }
      }
    }
    for (size_t j = 0; j < nb; ++j)
      if (!in[j]) throw Error(FV_ENOTSUP, "batched rules need bodies connected through shared variables");
  }
  u32 maxv = 0;
  for (u32 k = 0; k < n; ++k)
    for (auto& R : es[k]->rels_)
      for (u32 c = 0; c < R.arity; ++c) maxv = std::max(maxv, R.maxv[c]);
  const u64 stride = pow2_at_least(u64(maxv) + 1);
  if (stride * n > 0xFFFFFFFFull) throw Error(FV_ENOTSUP, "batched instances do not fit the 32-bit id space");

  auto B = std::make_shared<BatchResult>();
  fv_options mopt = E0.opt_;
  mopt.tuning = &E0.tune_;
  mopt.predictor = E0.learned_ ? E0.predictor_.data() : nullptr;
  if (!E0.trace_only_.empty()) mopt.trace_only = E0.trace_only_.c_str();
  B->merged = std::make_shared<Engine>(&mopt);
  B->stride = stride;
  Engine& M = *B->merged;
  M.allow_compaction_ = false;   // instances are sliced by id range afterwards
  for (auto& R : E0.rels_) M.relation_create(R.name.c_str(), R.arity);
  // one gather launch per relation concatenates every instance's staged facts
  std::vector<GatherDesc> desc(n);
  Buf ddesc = M.alloc(size_t(n) * sizeof(GatherDesc));
  try {
    for (size_t r = 0; r < M.rels_.size(); ++r) {
      Relation& D = M.rels_[r];
      u64 total = 0;
      for (u32 k = 0; k < n; ++k) {
        const Relation& S = es[k]->rels_[r];
        desc[k] = GatherDesc{{S.stage[0].as<u32>(), S.stage[1].as<u32>(), S.stage[2].as<u32>()}, S.staged, total,
                             u32(k * stride), 0};
        total += S.staged;
      }
      if (!total) continue;
      for (u32 k = 0; k < n; ++k) es[k]->sync();   // instance copies are ordered on their own streams
      for (u32 c = 0; c < D.arity; ++c) D.stage[c] = M.alloc(total * 4);
      M.hip(hipMemcpyAsync(ddesc.p, desc.data(), size_t(n) * sizeof(GatherDesc), hipMemcpyHostToDevice, M.stream_),
            "descriptor copy");
      u32* outs[3] = {D.stage[0].as<u32>(), D.stage[1].as<u32>(), D.stage[2].as<u32>()};
      M.launched(launch_gather_relabel(ddesc.as<GatherDesc>(), n, D.arity, outs, M.stream_), "gather");
      M.sync();   // the descriptor buffer is reused by the next relation
      D.staged = D.stage_cap = total;
      D.has_rows = true;
      for (u32 c = 0; c < D.arity; ++c) D.maxv[c] = u32(stride * n - 1);
    }
  } catch (...) {
    M.release(ddesc);
    throw;
  }
  M.release(ddesc);
  M.rules_ = E0.rules_;
  M.run(stats);
  B->deltas = M.deltas_;
  E0.trace_rows_ = M.trace_rows_;   // the merged run's join trace is reported on the first instance

  // every relation sorted once in the merged id space; instance k's rows are
  // the run whose first column lies in [k * stride, (k + 1) * stride)
  Buf bounds = M.alloc((size_t(n) + 1) * 8);
  try {
    B->cols.resize(M.rels_.size());
    B->bounds.resize(M.rels_.size());
    for (size_t r = 0; r < M.rels_.size(); ++r) {
      Relation& R = M.rels_[r];
      const u64 total = R.n_full;
      u32* outc[3] = {nullptr, nullptr, nullptr};
      for (u32 c = 0; c < R.arity; ++c) {
        B->cols[r].push_back(M.alloc(std::max<u64>(total, 1) * 4));
        outc[c] = B->cols[r][c].as<u32>();
      }
      u64 got = 0;
      if (total) M.export_rel(u32(r), outc, total, &got, true);
      B->bounds[r].assign(size_t(n) + 1, 0);
      M.launched(launch_bounds(outc[0], total, u32(stride), n, bounds.as<u64>(), M.stream_), "bounds");
      M.hip(hipMemcpyAsync(B->bounds[r].data(), bounds.p, (size_t(n) + 1) * 8, hipMemcpyDeviceToHost, M.stream_),
            "bounds readback");
      M.sync();
    }
  } catch (...) {
    M.release(bounds);
    throw;
  }
  M.release(bounds);
  for (u32 k = 0; k < n; ++k) {
    Engine& E = *es[k];
    E.batch_ = B;
    E.inst_ = k;
    E.ran_ = true;
    E.deltas_.clear();
    for (size_t r = 0; r < E.rels_.size(); ++r) {
      Relation& D = E.rels_[r];
      for (int c = 0; c < 3; ++c) E.release(D.stage[c]);
      D.staged = 0;
      D.n_full = B->bounds[r][k + 1] - B->bounds[r][k];
    }
  }
}

}  // namespace fv
