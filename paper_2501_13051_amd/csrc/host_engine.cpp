// Host evaluator (FV_HOST): the same plans and the same operators as the GPU
// path -- hash-index joins in two phases (Algorithm 1: count matches and
// prefix-sum them, then write every output at its offset), LSD radix sort of
// the packed new tuples, difference against full by a hash set of full's
// packed tuples, eager append to the contiguous columns of full -- run on host
// threads over host memory.  It is the counterpart of the paper's CPU variant
// of its engine (Section 5.3, Table 3: the same data structures on the CPU),
// selected explicitly; the GPU path never falls back to it.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>

#include <sched.h>

#include "engine.h"

namespace fv {

namespace {

u64 pow2_ge(u64 x) {
  u64 p = 1;
  while (p < x) p <<= 1;
  return p;
}

u64 hmix(u64 k) {   // MurmurHash3's 64-bit finalizer
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

}  // namespace

// A fixed set of worker threads; parallel_for hands out chunks of a range.
class HostPool {
 public:
  explicit HostPool(u32 n) : n_(std::max<u32>(1, n)) {
    for (u32 t = 1; t < n_; ++t) workers_.emplace_back([this, t] { loop(t); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& w : workers_) w.join();
  }
  u32 size() const { return n_; }
  // fn(begin, end, thread) over [0, n) in chunks of `grain`
  void parallel_for(u64 n, u64 grain, const std::function<void(u64, u64, u32)>& fn) {
    if (n == 0) return;
    grain = std::max<u64>(grain, 1);
    if (n <= grain || n_ == 1) { fn(0, n, 0); return; }
    {
      std::lock_guard<std::mutex> g(mu_);
      job_ = &fn;
      total_ = n;
      grain_ = grain;
      next_.store(0);
      busy_ = n_ - 1;
      ++gen_;
    }
    cv_.notify_all();
    run_chunks(0);
    std::unique_lock<std::mutex> g(mu_);
    done_cv_.wait(g, [&] { return busy_ == 0; });
    job_ = nullptr;
  }

 private:
  void run_chunks(u32 t) {
    for (;;) {
      const u64 b = next_.fetch_add(grain_);
      if (b >= total_) return;
      (*job_)(b, std::min(total_, b + grain_), t);
    }
  }
  void loop(u32 t) {
    u64 seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return gen_ != seen; });
        seen = gen_;
        if (stop_) return;
      }
      run_chunks(t);
      std::lock_guard<std::mutex> g(mu_);
      if (--busy_ == 0) done_cv_.notify_one();
    }
  }
  u32 n_;
  std::vector<std::thread> workers_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(u64, u64, u32)>* job_ = nullptr;
  u64 total_ = 0, grain_ = 1, gen_ = 0;
  std::atomic<u64> next_{0};
  u32 busy_ = 0;
  bool stop_ = false;
};

struct HostRel {
  std::vector<u32> stage[3];
  std::vector<u32> col[3];
  u64 n_full = 0, d_begin = 0;
  std::vector<u64> newk;
  std::vector<std::atomic<u64>> set;   // open addressing, all ones = empty
  u64 set_n = 0;
};

struct HostIndex {
  std::vector<Slot> table;
  std::vector<u32> perm;
  u64 mask = 0;
};

struct HostState {
  explicit HostState(u32 threads) : pool(threads) {}
  HostPool pool;
  std::vector<HostRel> rels;
  std::vector<HostIndex> idx;
  std::vector<std::vector<u32>> inter[kMaxCols];   // [col][inter id]
  std::vector<u64> inter_n;
};

namespace {

// LSD radix sort of (key, payload) pairs on the low `bits` bits of the key,
// 8-bit digits; per-thread digit counts, a prefix over (digit, thread), a
// stable scatter.  Keys and payloads end in a, b is scratch.
void radix_sort(HostPool& P, std::vector<u64>& a, std::vector<u32>* pa, u32 bits) {
  const u64 n = a.size();
  if (n < 2 || bits == 0) return;
  const u32 T = P.size();
  const u64 chunk = (n + T - 1) / T;
  std::vector<u64> b(n);
  std::vector<u32> pb(pa ? n : 0);
  std::vector<u64> cnt(size_t(T) * 256);
  for (u32 shift = 0; shift < bits; shift += 8) {
    std::fill(cnt.begin(), cnt.end(), 0);
    P.parallel_for(T, 1, [&](u64 t0, u64 t1, u32) {
      for (u64 t = t0; t < t1; ++t) {
        u64* c = &cnt[t * 256];
        for (u64 i = t * chunk; i < std::min(n, (t + 1) * chunk); ++i) ++c[(a[i] >> shift) & 255];
      }
    });
    u64 sum = 0;
    for (u32 d = 0; d < 256; ++d)
      for (u32 t = 0; t < T; ++t) {
        const u64 c = cnt[size_t(t) * 256 + d];
        cnt[size_t(t) * 256 + d] = sum;
        sum += c;
      }
    P.parallel_for(T, 1, [&](u64 t0, u64 t1, u32) {
      for (u64 t = t0; t < t1; ++t) {
        u64* c = &cnt[t * 256];
        for (u64 i = t * chunk; i < std::min(n, (t + 1) * chunk); ++i) {
          const u64 pos = c[(a[i] >> shift) & 255]++;
          b[pos] = a[i];
          if (pa) pb[pos] = (*pa)[i];
        }
      }
    });
    a.swap(b);
    if (pa) pa->swap(pb);
  }
}

u32 bits_of(u64 x) {
  u32 b = 0;
  while (x) { ++b; x >>= 1; }
  return b;
}

bool set_insert(std::vector<std::atomic<u64>>& set, u64 key) {   // true: newly inserted
  const u64 mask = set.size() - 1;
  for (u64 h = hmix(key) & mask;; h = (h + 1) & mask) {
    u64 cur = set[h].load(std::memory_order_relaxed);
    if (cur == key) return false;
    if (cur == kEmptyKey) {
      if (set[h].compare_exchange_strong(cur, key, std::memory_order_relaxed)) return true;
      if (cur == key) return false;
    }
  }
}

}  // namespace

u32 Engine::host_threads() {
  cpu_set_t s;
  if (sched_getaffinity(0, sizeof(s), &s) == 0) return u32(std::max(1, CPU_COUNT(&s)));
  return std::max(1u, std::thread::hardware_concurrency());
}

void Engine::host_load(u32 rel, const u32* const* cols, u64 n, bool on_device) {
  if (!host_) host_ = std::make_shared<HostState>(host_threads_);
  if (host_->rels.size() < rels_.size()) host_->rels.resize(rels_.size());
  Relation& R = rels_[rel];
  HostRel& H = host_->rels[rel];
  std::vector<u32> in[3];
  u32 mx[3] = {0, 0, 0};
  for (u32 c = 0; c < R.arity; ++c) {
    in[c].resize(n);
    if (on_device) hip(hipMemcpy(in[c].data(), cols[c], n * 4, hipMemcpyDeviceToHost), "load copy");
    else std::memcpy(in[c].data(), cols[c], n * 4);
    for (u64 i = 0; i < n; ++i) mx[c] = std::max(mx[c], in[c][i]);
    if (mx[c] == 0xFFFFFFFFu) throw Error(FV_ERESERVED, "value 0xFFFFFFFF is reserved");
  }
  for (u32 c = 0; c < R.arity; ++c) {
    H.stage[c].insert(H.stage[c].end(), in[c].begin(), in[c].end());
    R.maxv[c] = std::max(R.maxv[c], mx[c]);
    R.lmax[c] = std::max(R.lmax[c], mx[c]);
  }
  R.staged += n;
  R.has_rows = true;
}

// Index of rows [0, n_full) of its relation that pass its filters: rows
// sorted by key (radix sort of (key, row)), one table slot per distinct key
// with its run in perm -- the layout of the GPU index.
void Engine::host_build_index(u32 i) {
  const Index& ix = indices_[i];
  const HostRel& H = host_->rels[ix.rel];
  HostIndex& X = host_->idx[i];
  HostPool& P = host_->pool;
  const u64 n = H.n_full;
  std::vector<u64> keys;
  std::vector<u32> rows;
  keys.reserve(n);
  rows.reserve(n);
  for (u64 r = 0; r < n; ++r) {
    bool ok = true;
    for (u32 f = 0; f < ix.nfilt; ++f) ok = ok && H.col[ix.fcol[f]][r] == ix.fval[f];
    if (!ok) continue;
    const u64 a = H.col[ix.keycol[0]][r];
    keys.push_back(ix.nkey == 2 ? (a << 32) | H.col[ix.keycol[1]][r] : a);
    rows.push_back(u32(r));
  }
  const u32 kb = ix.nkey == 2 ? 32 + bits_of(rels_[ix.rel].maxv[ix.keycol[1]]) : bits_of(rels_[ix.rel].maxv[ix.keycol[0]]);
  radix_sort(P, keys, &rows, ix.nkey == 2 ? 64 : std::max<u32>(kb, 1));
  u64 ndv = 0;
  for (u64 j = 0; j < keys.size(); ++j) ndv += (j == 0 || keys[j] != keys[j - 1]);
  const u64 cap = pow2_ge(std::max<u64>(2 * ndv, 64));
  X.table.assign(cap, Slot{kEmptyKey, 0, 0});
  X.mask = cap - 1;
  for (u64 j = 0; j < keys.size();) {
    u64 e = j;
    while (e < keys.size() && keys[e] == keys[j]) ++e;
    u64 h = hmix(keys[j]) & X.mask;
    while (X.table[h].key != kEmptyKey) h = (h + 1) & X.mask;
    X.table[h] = Slot{keys[j], u32(j), u32(e - j)};
    j = e;
  }
  X.perm.swap(rows);
}

// One plan: its joins run probe side by probe side, each in two phases per
// chunk of probe rows (count the outputs that pass the filters, prefix-sum
// the chunk counts, write each output at its offset).
void Engine::host_exec_plan(Plan& p) {
  HostState& S = *host_;
  HostPool& P = S.pool;
  const bool initial = p.delta_pos < 0;
  for (size_t k = 0; k < p.steps.size(); ++k) {
    Step& s = p.steps[k];
    const u32* pcol[kMaxCols] = {};
    u64 pb = 0, pe = 0;
    if (k == 0) {
      const HostRel& H = S.rels[p.src_rel];
      for (u32 c = 0; c < rels_[p.src_rel].arity; ++c) pcol[c] = H.col[c].data();
      pb = initial ? 0 : H.d_begin;
      pe = H.n_full;
    } else {
      const int ib = p.steps[k - 1].out_buf;
      for (u32 c = 0; c < inters_[ib].ncols; ++c) pcol[c] = S.inter[c][ib].data();
      pe = S.inter_n[ib];
    }
    const u32* bcol[3] = {};
    u64 nbuild = 0;
    const HostIndex* X = nullptr;
    if (!s.select_only) {
      const HostRel& B = S.rels[s.brel];
      for (u32 c = 0; c < rels_[s.brel].arity; ++c) bcol[c] = B.col[c].data();
      nbuild = B.n_full;
      if (s.index != kNoIndex) X = &S.idx[s.index];
    }
    auto val = [&](const Src& src, u64 prow, u64 brow) -> u32 {
      if (src.kind == kSrcConst) return src.v;
      if (src.kind == kSrcProbe) return pcol[src.v][prow];
      return bcol[src.v][brow];
    };
    auto probe_ok = [&](u64 r) {
      for (auto& f : s.pf) {
        const u32 a = val(f.a, r, 0), b = val(f.b, r, 0);
        if (f.op == kEq ? a != b : a == b) return false;
      }
      return true;
    };
    auto run_of = [&](u64 r, u64& st, u64& cnt) {
      if (s.select_only) { st = 0; cnt = 1; return; }
      if (!X) { st = 0; cnt = nbuild; return; }
      const u64 a = val(s.key[0], r, 0);
      const u64 key = s.nkey == 2 ? (a << 32) | val(s.key[1], r, 0) : a;
      st = cnt = 0;
      for (u64 h = hmix(key) & X->mask;; h = (h + 1) & X->mask) {
        const Slot& sl = X->table[h];
        if (sl.key == key) { st = sl.start; cnt = sl.count; return; }
        if (sl.key == kEmptyKey) return;
      }
    };
    auto keep = [&](u64 r, u64 brow) {
      for (auto& f : s.wf) {
        const u32 a = val(f.a, r, brow), b = val(f.b, r, brow);
        if (f.op == kEq ? a != b : a == b) return false;
      }
      return true;
    };
    const u64 n = pe - pb;
    const u64 grain = 4096;
    const u64 nchunks = (n + grain - 1) / grain;
    std::vector<u64> off(nchunks + 1, 0);
    // phase 1: outputs per chunk
    P.parallel_for(nchunks, 1, [&](u64 c0, u64 c1, u32) {
      for (u64 c = c0; c < c1; ++c) {
        u64 m = 0;
        for (u64 r = pb + c * grain; r < std::min(pe, pb + (c + 1) * grain); ++r) {
          if (!probe_ok(r)) continue;
          u64 st, cnt;
          run_of(r, st, cnt);
          for (u64 i = 0; i < cnt; ++i) {
            const u64 brow = s.select_only ? 0 : (X ? X->perm[st + i] : i);
            m += keep(r, brow) ? 1 : 0;
          }
        }
        off[c + 1] = m;
      }
    });
    for (u64 c = 0; c < nchunks; ++c) off[c + 1] += off[c];
    const u64 total = off[nchunks];
    join_out_ += s.select_only ? 0 : total;
    // phase 2: write at the offsets
    const bool to_head = s.out_buf < 0;
    u64 base = 0;
    u64* keys = nullptr;
    u32* ocol[kMaxCols] = {};
    const Relation& HR = rels_[s.head_rel];
    if (to_head) {
      HostRel& H = S.rels[s.head_rel];
      base = H.newk.size();
      H.newk.resize(base + total);
      keys = H.newk.data();
    } else {
      for (u32 c = 0; c < s.out.size(); ++c) {
        S.inter[c][s.out_buf].resize(total);
        ocol[c] = S.inter[c][s.out_buf].data();
      }
      S.inter_n[s.out_buf] = total;
    }
    P.parallel_for(nchunks, 1, [&](u64 c0, u64 c1, u32) {
      for (u64 c = c0; c < c1; ++c) {
        u64 pos = off[c];
        for (u64 r = pb + c * grain; r < std::min(pe, pb + (c + 1) * grain); ++r) {
          if (!probe_ok(r)) continue;
          u64 st, cnt;
          run_of(r, st, cnt);
          for (u64 i = 0; i < cnt; ++i) {
            const u64 brow = s.select_only ? 0 : (X ? X->perm[st + i] : i);
            if (!keep(r, brow)) continue;
            if (to_head) {
              u64 key = 0;
              for (u32 o = 0; o < s.out.size(); ++o) key |= u64(val(s.out[o], r, brow)) << HR.shift[o];
              keys[base + pos] = key;
            } else {
              for (u32 o = 0; o < s.out.size(); ++o) ocol[o][pos] = val(s.out[o], r, brow);
            }
            ++pos;
          }
        }
      }
    });
  }
}

// Sort the relation's new keys, drop repeats and tuples already in full
// (insert-if-absent into full's tuple set), append the survivors in order.
u64 Engine::host_finish_relation(u32 ri) {
  HostState& S = *host_;
  HostPool& P = S.pool;
  Relation& R = rels_[ri];
  HostRel& H = S.rels[ri];
  std::vector<u64>& k = H.newk;
  radix_sort(P, k, nullptr, R.bits);
  const u64 n = k.size();
  // the set holds full plus this round's survivors; keep its load below 1/2
  if (2 * (H.n_full + n) > H.set.size()) {
    const u64 cap = pow2_ge(std::max<u64>(4 * (H.n_full + n), 1024));
    std::vector<std::atomic<u64>> ns(cap);
    for (auto& x : ns) x.store(kEmptyKey, std::memory_order_relaxed);
    H.set.swap(ns);
    P.parallel_for(H.n_full, 65536, [&](u64 b, u64 e, u32) {
      for (u64 r = b; r < e; ++r) {
        u64 key = 0;
        for (u32 c = 0; c < R.arity; ++c) key |= u64(H.col[c][r]) << R.shift[c];
        set_insert(H.set, key);
      }
    });
  }
  const u64 grain = 65536;
  const u64 nchunks = (n + grain - 1) / grain;
  std::vector<uint8_t> surv(n, 0);
  std::vector<u64> off(nchunks + 1, 0);
  P.parallel_for(nchunks, 1, [&](u64 c0, u64 c1, u32) {
    for (u64 c = c0; c < c1; ++c) {
      u64 m = 0;
      for (u64 i = c * grain; i < std::min(n, (c + 1) * grain); ++i) {
        if (i > 0 && k[i] == k[i - 1]) continue;
        if (set_insert(H.set, k[i])) { surv[i] = 1; ++m; }
      }
      off[c + 1] = m;
    }
  });
  for (u64 c = 0; c < nchunks; ++c) off[c + 1] += off[c];
  const u64 d = off[nchunks];
  for (u32 c = 0; c < R.arity; ++c) H.col[c].resize(H.n_full + d);
  P.parallel_for(nchunks, 1, [&](u64 c0, u64 c1, u32) {
    for (u64 c = c0; c < c1; ++c) {
      u64 pos = H.n_full + off[c];
      for (u64 i = c * grain; i < std::min(n, (c + 1) * grain); ++i) {
        if (!surv[i]) continue;
        for (u32 col = 0; col < R.arity; ++col) {
          const u64 m = R.width[col] >= 32 ? 0xFFFFFFFFull : ((1ull << R.width[col]) - 1);
          H.col[col][pos] = u32((k[i] >> R.shift[col]) & m);
        }
        ++pos;
      }
    }
  });
  k.clear();
  return d;
}

// The loaded facts' column bounds under condition sets (the layout of
// launch_cond_bounds), on the host.
void Engine::host_fact_bounds(u32 rel, const CondSet* q, u32 nq, u32* out) {
  const Relation& R = rels_[rel];
  const HostRel& H = host_->rels[rel];
  for (u32 i = 0; i < nq * 8; ++i) out[i] = (i % 8) < 3 ? 0xFFFFFFFFu : 0u;
  for (u64 r = 0; r < R.staged; ++r)
    for (u32 k = 0; k < nq; ++k) {
      bool ok = true;
      for (u32 i = 0; i < q[k].n; ++i) ok = ok && H.stage[q[k].col[i]][r] == q[k].val[i];
      if (!ok) continue;
      out[k * 8 + 6] = 1;
      for (u32 c = 0; c < R.arity; ++c) {
        out[k * 8 + c] = std::min(out[k * 8 + c], H.stage[c][r]);
        out[k * 8 + 3 + c] = std::max(out[k * 8 + 3 + c], H.stage[c][r]);
      }
    }
}

void Engine::run_host(fv_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!host_) host_ = std::make_shared<HostState>(host_threads_);
  HostState& S = *host_;
  S.rels.resize(rels_.size());
  fit_packing();
  plan_all();
  S.idx.assign(indices_.size(), HostIndex{});
  for (auto& v : S.inter) v.assign(inters_.size(), {});
  S.inter_n.assign(inters_.size(), 0);
  // ingest: pack, sort, unique (relations are sets)
  for (u32 ri = 0; ri < rels_.size(); ++ri) {
    Relation& R = rels_[ri];
    HostRel& H = S.rels[ri];
    const u64 n = R.staged;
    H.newk.resize(n);
    for (u64 i = 0; i < n; ++i) {
      u64 key = 0;
      for (u32 c = 0; c < R.arity; ++c) key |= u64(H.stage[c][i]) << R.shift[c];
      H.newk[i] = key;
    }
    for (auto& st : H.stage) std::vector<u32>().swap(st);
    host_finish_relation(ri);
    H.d_begin = 0;
    H.n_full = H.col[0].size();
    R.n_full = H.n_full;
    R.seeds = H.n_full;
    R.staged = 0;
    if (!R.used_as_head) std::vector<std::atomic<u64>>().swap(H.set);   // loaded relations need no set
  }
  for (u32 i = 0; i < indices_.size(); ++i) host_build_index(i);
  deltas_.clear();
  join_out_ = 0;
  for (bool initial = true;; initial = false) {
    for (auto& p : initial ? init_plans_ : delta_plans_)
      if (initial || S.rels[p.src_rel].n_full > S.rels[p.src_rel].d_begin) host_exec_plan(p);
    u64 total = 0;
    std::vector<u64> d(rels_.size(), 0);
    for (u32 ri = 0; ri < rels_.size(); ++ri)
      if (rels_[ri].used_as_head) d[ri] = host_finish_relation(ri);
    for (u32 ri = 0; ri < rels_.size(); ++ri) {
      HostRel& H = S.rels[ri];
      if (rels_[ri].used_as_head) {
        H.d_begin = H.n_full;
        H.n_full += d[ri];
        total += d[ri];
      } else {
        H.d_begin = H.n_full;   // loaded relations never have a delta
      }
      rels_[ri].n_full = H.n_full;
    }
    deltas_.push_back(total);
    if (total == 0) break;
    for (u32 i = 0; i < indices_.size(); ++i)
      if (rels_[indices_[i].rel].used_as_head) host_build_index(i);
  }
  const auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    *stats = fv_stats{};
    stats->iterations = u32(deltas_.size());
    u64 derived = 0;
    for (auto& R : rels_)
      if (R.used_as_head) derived += R.n_full - R.seeds;
    stats->derived_tuples = derived;
    stats->join_output_tuples = join_out_;
    stats->ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
}

// The host side of value compaction: sorted distinct values of the loaded
// columns and rule constants, and the loaded columns rewritten as ranks.
void Engine::host_compact_values() {
  HostState& S = *host_;
  std::vector<u64> v;
  for (auto& r : rules_) {
    for (auto& t : r.head.t) if (t.is_const) v.push_back(t.value);
    for (auto& a : r.body) for (auto& t : a.t) if (t.is_const) v.push_back(t.value);
  }
  for (u32 ri = 0; ri < rels_.size(); ++ri)
    for (u32 c = 0; c < rels_[ri].arity; ++c) v.insert(v.end(), S.rels[ri].stage[c].begin(), S.rels[ri].stage[c].end());
  radix_sort(S.pool, v, nullptr, 32);
  dict_host_.clear();
  for (u64 i = 0; i < v.size(); ++i)
    if (i == 0 || v[i] != v[i - 1]) dict_host_.push_back(u32(v[i]));
  std::vector<u64>().swap(v);
  for (u32 ri = 0; ri < rels_.size(); ++ri)
    for (u32 c = 0; c < rels_[ri].arity; ++c) {
      std::vector<u32>& col = S.rels[ri].stage[c];
      S.pool.parallel_for(col.size(), 1 << 16, [&](u64 b, u64 e, u32) {
        for (u64 i = b; i < e; ++i)
          col[i] = u32(std::lower_bound(dict_host_.begin(), dict_host_.end(), col[i]) - dict_host_.begin());
      });
    }
}

void Engine::host_export(u32 rel, u32* const* cols, u64 n, bool on_device) {
  const Relation& R = rels_[rel];
  const HostRel& H = host_->rels[rel];
  std::vector<u64> k(n);
  for (u64 i = 0; i < n; ++i) {
    u64 key = 0;
    for (u32 c = 0; c < R.arity; ++c) key |= u64(H.col[c][i]) << R.shift[c];
    k[i] = key;
  }
  radix_sort(host_->pool, k, nullptr, R.bits);
  std::vector<u32> out(n);
  for (u32 c = 0; c < R.arity; ++c) {
    const u64 m = R.width[c] >= 32 ? 0xFFFFFFFFull : ((1ull << R.width[c]) - 1);
    for (u64 i = 0; i < n; ++i) out[i] = u32((k[i] >> R.shift[c]) & m);
    if (compacted_)
      for (u64 i = 0; i < n; ++i) out[i] = dict_host_[out[i]];
    if (on_device) hip(hipMemcpy(cols[c], out.data(), n * 4, hipMemcpyHostToDevice), "export copy");
    else std::memcpy(cols[c], out.data(), n * 4);
  }
}

}  // namespace fv
