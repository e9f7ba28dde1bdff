// Per-subset power-trace schedules ("chain programs").
//
// For a subset matrix M (d x d) the coefficient c_k needs t_j = tr(M^j) for j = 1..k. A set of
// powers P (an addition chain: 1 in P, every other element the sum of two earlier ones) is formed
// with |P| - 1 matrix products; every j is then either in P (a diagonal trace, d flops) or a sum
// p_a + p_b of two elements (an inner product tr(M^a M^b), d^2 complex multiply-adds). The search
// below picks the chain with the fewest products whose live powers fit in a given number of LDS
// slots, then the fewest slots, then the fewest inner products.
#include <algorithm>
#include <cstring>
#include <vector>

#include "gbs_internal.h"

namespace gbs {
namespace {

struct Candidate {
  std::vector<int> P;
  std::vector<std::pair<int, int>> src;  // src[i] = (a, b): P[i] = P[a] + P[b]
};

struct Sched {
  bool ok = false;
  int nmul = 0, nslots = 0, npair = 0;
  ChainProgram prog{};
};

// Turn a chain into a program; returns ok=false if some t_j cannot be formed or slots overflow.
Sched schedule(const Candidate& c, int k, int slot_limit) {
  Sched r;
  const int np = (int)c.P.size();
  // trace sources: step, a, b (b = -1 for a diagonal)
  struct Tr {
    int step, a, b;
  };
  std::vector<Tr> tr(k + 1, Tr{-1, -1, -1});
  for (int j = 1; j <= k; ++j) {
    for (int i = 0; i < np; ++i)
      if (c.P[i] == j) tr[j] = Tr{i, i, -1};  // a formed power: read its diagonal
    for (int i = 0; i < np && tr[j].step < 0; ++i)
      for (int a = 0; a <= i; ++a)
        if (c.P[a] + c.P[i] == j) {  // earliest inner product that gives it
          tr[j] = Tr{i, a, i};
          break;
        }
    if (tr[j].step < 0) return r;
  }
  std::vector<int> last_tr(np, -1), last_mul(np, -1);
  for (int j = 1; j <= k; ++j) {
    last_tr[tr[j].a] = std::max(last_tr[tr[j].a], tr[j].step);
    if (tr[j].b >= 0) last_tr[tr[j].b] = std::max(last_tr[tr[j].b], tr[j].step);
  }
  for (int i = 1; i < np; ++i) {
    last_mul[c.src[i].first] = std::max(last_mul[c.src[i].first], i);
    last_mul[c.src[i].second] = std::max(last_mul[c.src[i].second], i);
  }
  // slot assignment
  std::vector<int> slot_of(np, -1);
  std::vector<int> holder(kMaxSlots, -1);  // power index held by each slot
  slot_of[0] = 0;
  holder[0] = 0;
  int used = 1;
  ChainProgram& pg = r.prog;
  pg.nops = 0;
  auto emit = [&](uint8_t t, int x, int a, int b) -> bool {
    if (pg.nops >= kMaxOps) return false;
    pg.ops[pg.nops++] = Op{t, (uint8_t)x, (uint8_t)a, (uint8_t)b};
    return true;
  };
  auto emit_traces = [&](int step) -> bool {
    for (int j = 1; j <= k; ++j) {
      if (tr[j].step != step) continue;
      if (tr[j].b < 0) {
        if (!emit(OP_TDIAG, j, slot_of[tr[j].a], 0)) return false;
      } else {
        if (!emit(OP_TPAIR, j, slot_of[tr[j].a], slot_of[tr[j].b])) return false;
        r.npair++;
      }
    }
    return true;
  };
  auto last_use = [&](int q) { return std::max(last_mul[q], last_tr[q]); };
  if (!emit_traces(0)) return r;
  for (int i = 1; i < np; ++i) {
    // release powers no longer needed at or after this step
    int reuse = -1;
    for (int sl = 0; sl < kMaxSlots; ++sl) {
      int q = holder[sl];
      if (q < 0) continue;
      if (last_use(q) < i) holder[sl] = -1;  // dead before this step
      else if (last_use(q) == i && last_tr[q] < i && reuse < 0) reuse = sl;  // dies as an operand here
    }
    int dst = reuse;
    if (dst < 0)
      for (int sl = 0; sl < kMaxSlots; ++sl)
        if (holder[sl] < 0) {
          dst = sl;
          break;
        }
    if (dst < 0 || dst >= slot_limit) return r;
    if (!emit(OP_MUL, dst, slot_of[c.src[i].first], slot_of[c.src[i].second])) return r;
    r.nmul++;
    if (reuse >= 0) slot_of[holder[reuse]] = -1;
    holder[dst] = i;
    slot_of[i] = dst;
    int cnt = 0;
    for (int sl = 0; sl < kMaxSlots; ++sl) cnt += holder[sl] >= 0;
    used = std::max(used, std::max(cnt, dst + 1));
    if (!emit_traces(i)) return r;
  }
  r.nslots = used;
  r.ok = true;
  pg.nslots = used;
  pg.nmul = r.nmul;
  pg.npair = r.npair;
  return r;
}

void dfs(Candidate& c, int k, int maxlen, int slot_limit, Sched& best) {
  Sched s = schedule(c, k, slot_limit);
  if (s.ok) {
    auto key = [](const Sched& x) { return std::make_tuple(x.nmul, x.nslots, x.npair); };
    if (!best.ok || key(s) < key(best)) best = s;
    return;
  }
  if ((int)c.P.size() >= maxlen) return;
  if (best.ok && (int)c.P.size() - 1 >= best.nmul) return;  // adding a power cannot beat best
  std::vector<std::pair<int, std::pair<int, int>>> cand;
  for (int a = 0; a < (int)c.P.size(); ++a)
    for (int b = a; b < (int)c.P.size(); ++b) {
      int v = c.P[a] + c.P[b];
      if (v <= c.P.back() || v > k) continue;
      bool dup = false;
      for (auto& e : cand) dup |= e.first == v;
      if (!dup) cand.push_back({v, {a, b}});
    }
  std::sort(cand.begin(), cand.end());
  for (auto& e : cand) {
    c.P.push_back(e.first);
    c.src.push_back(e.second);
    dfs(c, k, maxlen, slot_limit, best);
    c.P.pop_back();
    c.src.pop_back();
  }
}

}  // namespace

// Best chain program for k with at most slot_limit LDS slots; returns false if none was found.
bool build_chain_program(int k, int slot_limit, ChainProgram* out) {
  Sched best;
  for (int maxlen = 1; maxlen <= 12 && !best.ok; ++maxlen) {
    Candidate c;
    c.P = {1};
    c.src = {{0, 0}};
    dfs(c, k, maxlen, slot_limit, best);
  }
  if (!best.ok) return false;
  *out = best.prog;
  return true;
}

}  // namespace gbs
