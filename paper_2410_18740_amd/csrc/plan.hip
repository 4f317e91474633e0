// Contraction planner and executor for the effective operator of a one- or
// two-site window of the MPO, and for environment updates.
//
// Every core entry is a combination of the local operators {I, X, P, S, X^2,
// XP + PX} (coefficient vector c); the window operator is therefore
//   O[l][n] = sum_{a,b} c_{l n a b} op_a (x) op_b,
// with l a left-environment channel and n a right-environment channel.  The
// planner turns these terms into
//   Y_c   = Lmix_c * theta                      (batched MFMA GEMM, K = chi_l)
//   T_j   = sum coef * (op_a (x) op_b) Y_c       (memory-bound operator kernel)
//   theta' = sum_r src_r * Rmix_r^T               (chained-K MFMA GEMM, split-K)
// where pass-through channels alias Y buffers (no copy), channels fed by many
// left channels with the identity (the dense scalar block of the middle core)
// are folded into mixed left environments, and an operator applied to one
// source but needed by many right channels is folded into one mixed right
// environment.  This keeps the memory-bound stage to a handful of buffers.
#include <algorithm>
#include <map>
#include <set>
#include <tuple>
#include <cstring>
#include "internal.h"

std::vector<Term2> window_terms(const tn_mpo* mpo, int site, int nsites) {
  std::map<std::tuple<int, int, int, int>, double> acc;
  if (nsites == 1) {
    for (const auto& e : mpo->entries[site])
      for (int a = 0; a <= NOPS; ++a)
        if (e.c[a] != 0.0) acc[{e.row, e.col, a, 0}] += e.c[a];
  } else {
    const auto& E1 = mpo->entries[site];
    const auto& E2 = mpo->entries[site + 1];
    std::map<int, std::vector<const CoreEntry*>> by_row;
    for (const auto& e : E2) by_row[e.row].push_back(&e);
    for (const auto& e1 : E1) {
      auto it = by_row.find(e1.col);
      if (it == by_row.end()) continue;
      for (const CoreEntry* e2 : it->second)
        for (int a = 0; a <= NOPS; ++a) {
          if (e1.c[a] == 0.0) continue;
          for (int b = 0; b <= NOPS; ++b) {
            if (e2->c[b] == 0.0) continue;
            acc[{e1.row, e2->col, a, b}] += e1.c[a] * e2->c[b];
          }
        }
    }
  }
  std::vector<Term2> out;
  for (auto& kv : acc) {
    if (kv.second == 0.0) continue;
    out.push_back({std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first), kv.second});
  }
  return out;
}

Plan build_plan(const std::vector<Term2>& terms, int wl, int wr, bool allow_right_fold) {
  (void)wl; (void)wr;
  Plan P;
  std::map<int, std::vector<std::pair<int, double>>> II;
  std::vector<Term2> ops;
  for (const auto& t : terms) {
    if (t.a == 0 && t.b == 0) II[t.n].push_back({t.l, t.c});
    else ops.push_back(t);
  }
  std::map<int, int> orig;
  auto ych_orig = [&](int l) {
    auto it = orig.find(l);
    if (it != orig.end()) return it->second;
    PlanL L;
    L.src.push_back({l, 1.0});
    P.L.push_back(L);
    orig[l] = (int)P.L.size() - 1;
    return (int)P.L.size() - 1;
  };
  std::vector<bool> used(ops.size(), false);
  if (allow_right_fold) {
    std::map<std::tuple<int, int, int>, std::vector<int>> g;
    for (size_t i = 0; i < ops.size(); ++i) g[{ops[i].l, ops[i].a, ops[i].b}].push_back((int)i);
    for (auto& kv : g) {
      std::set<int> ns;
      for (int i : kv.second) ns.insert(ops[i].n);
      if (ns.size() < 2) continue;
      PlanT tj;
      tj.terms.push_back({ych_orig(std::get<0>(kv.first)), std::get<1>(kv.first), std::get<2>(kv.first), 1.0});
      P.T.push_back(tj);
      PlanR r;
      r.kind = 1;
      r.idx = (int)P.T.size() - 1;
      for (int i : kv.second) { r.env.push_back({ops[i].n, ops[i].c}); used[i] = true; }
      P.R.push_back(r);
    }
  }
  std::map<int, std::vector<PlanTerm>> tterms;
  {
    std::map<std::tuple<int, int, int>, std::vector<int>> g;
    for (size_t i = 0; i < ops.size(); ++i)
      if (!used[i]) g[{ops[i].n, ops[i].a, ops[i].b}].push_back((int)i);
    for (auto& kv : g) {
      const int n = std::get<0>(kv.first), a = std::get<1>(kv.first), b = std::get<2>(kv.first);
      if (kv.second.size() >= 2) {
        PlanL L;
        for (int i : kv.second) L.src.push_back({ops[i].l, ops[i].c});
        P.L.push_back(L);
        tterms[n].push_back({(int)P.L.size() - 1, a, b, 1.0});
      } else {
        const int i = kv.second[0];
        tterms[n].push_back({ych_orig(ops[i].l), a, b, ops[i].c});
      }
    }
  }
  std::set<int> targets;
  for (auto& kv : II) targets.insert(kv.first);
  for (auto& kv : tterms) targets.insert(kv.first);
  for (int n : targets) {
    int ii = -1;
    auto it = II.find(n);
    if (it != II.end()) {
      if (it->second.size() == 1 && it->second[0].second == 1.0) ii = ych_orig(it->second[0].first);
      else {
        PlanL L;
        L.src = it->second;
        P.L.push_back(L);
        ii = (int)P.L.size() - 1;
      }
    }
    auto jt = tterms.find(n);
    if (jt != tterms.end()) {
      PlanT tj;
      if (ii >= 0) tj.terms.push_back({ii, 0, 0, 1.0});
      for (auto& t : jt->second) tj.terms.push_back(t);
      P.T.push_back(tj);
      P.R.push_back({1, (int)P.T.size() - 1, {{n, 1.0}}});
    } else {
      P.R.push_back({0, ii, {{n, 1.0}}});
    }
  }
  return P;
}

// ------------------------------------------------------------------ window executor
static bool is_plain(const std::vector<std::pair<int, double>>& v) { return v.size() == 1 && v[0].second == 1.0; }

void WindowOp::setup(tn_ctx* c, const tn_mpo* mpo, int site, int nsites, int prec_, int chi_l_, int chi_r_,
                     const std::vector<const void*>& envL, const std::vector<const void*>& envRt, bool raw_leg0,
                     const std::string& tag) {
  ctx = c;
  prec = prec_;
  chi_l = chi_l_;
  chi_r = chi_r_;
  ds = raw_leg0 ? mpo->D_raw : mpo->d;
  dt = (nsites == 2) ? mpo->d : 1;
  const int wl = mpo->w[site], wr = mpo->w[site + nsites];
  auto terms = window_terms(mpo, site, nsites);
  plan = build_plan(terms, wl, wr, true);
  const size_t eb = elem_bytes(prec);
  n = (size_t)chi_l * ds * dt * chi_r;
  const int gprec = prec;  // GEMM form
  const int sprec = (prec == PREC_FP64) ? PREC_FP64 : PREC_FP32;  // storage form
  // --- mixed left environments
  std::vector<const void*> Lptr(plan.L.size());
  std::vector<MixJob> mixjobs;
  std::vector<MixTerm> mixterms;
  int nLmix = 0;
  for (auto& L : plan.L) nLmix += is_plain(L.src) ? 0 : 1;
  int nRmix = 0;
  for (auto& R : plan.R) nRmix += is_plain(R.env) ? 0 : 1;
  char* Lmix = (char*)ws_get(ctx, tag + ":Lmix", std::max<size_t>(1, nLmix) * chi_l * chi_l * eb);
  char* Rmix = (char*)ws_get(ctx, tag + ":Rmix", std::max<size_t>(1, nRmix) * chi_r * chi_r * eb);
  int il = 0;
  for (size_t i = 0; i < plan.L.size(); ++i) {
    auto& L = plan.L[i];
    if (is_plain(L.src)) { Lptr[i] = envL[L.src[0].first]; continue; }
    void* dst = Lmix + (size_t)il * chi_l * chi_l * eb;
    ++il;
    mixjobs.push_back({dst, (int)mixterms.size(), (int)L.src.size()});
    for (auto& s : L.src) mixterms.push_back({envL[s.first], s.second});
    Lptr[i] = dst;
  }
  std::vector<MixJob> mixjobsR;
  std::vector<const void*> Rptr(plan.R.size());
  int ir = 0;
  for (size_t i = 0; i < plan.R.size(); ++i) {
    auto& R = plan.R[i];
    if (is_plain(R.env)) { Rptr[i] = envRt[R.env[0].first]; continue; }
    void* dst = Rmix + (size_t)ir * chi_r * chi_r * eb;
    ++ir;
    mixjobsR.push_back({dst, (int)mixterms.size(), (int)R.env.size()});
    for (auto& s : R.env) mixterms.push_back({envRt[s.first], s.second});
    Rptr[i] = dst;
  }
  // --- buffers
  char* Y = (char*)ws_get(ctx, tag + ":Y", std::max<size_t>(1, plan.L.size()) * n * eb);
  char* T = (char*)ws_get(ctx, tag + ":T", std::max<size_t>(1, plan.T.size()) * n * eb);
  xin = ws_get(ctx, tag + ":xin", n * eb);
  ybuf = Y;
  rptr = Rptr;
  // split-K for the right contraction: as many splits as fill one round of
  // workgroups (the GEMM's tiles at its workgroups per CU on 256 CUs) without
  // starting a second, partly filled round
  const int BMr = (gprec == PREC_FP64) ? 64 : 128, BNr = 64;
  const int round = 256 * (gprec == PREC_FP32 ? 3 : 2);
  const int Mr = chi_l * ds * dt;
  const int tiles = ((Mr + BMr - 1) / BMr) * ((chi_r + BNr - 1) / BNr);
  const int nR = (int)plan.R.size();
  nsplit = std::max(1, std::min(nR, round / tiles));
  partials = ws_get(ctx, tag + ":part", (size_t)nsplit * n * eb);
  // --- descriptors
  std::vector<GemmJob> jl;
  std::vector<GemmSeg> sl;
  for (size_t i = 0; i < plan.L.size(); ++i) {
    sl.push_back({Lptr[i], xin, chi_l, (int64_t)ds * dt * chi_r, chi_l, 0});
    jl.push_back({Y + i * n * eb, (int64_t)ds * dt * chi_r, chi_l, ds * dt * chi_r, (int)sl.size() - 1, 1});
  }
  std::vector<OpJob> oj;
  std::vector<OpTerm> ot;
  for (size_t j = 0; j < plan.T.size(); ++j) {
    OpJob job{T + j * n * eb, (int)ot.size(), (int)plan.T[j].terms.size(), 0, 0};
    for (auto& t : plan.T[j].terms) {
      const void* oA = (t.a == 0) ? nullptr : mpo->op_ptr(sprec, site, t.a, raw_leg0);
      const void* oB = (t.b == 0) ? nullptr : mpo->op_ptr(sprec, site + 1, t.b, false);
      ot.push_back({Y + (size_t)t.ych * n * eb, oA, oB, t.c});
    }
    oj.push_back(job);
  }
  std::vector<GemmJob> jr;
  std::vector<GemmSeg> sr;
  for (int g = 0; g < nsplit; ++g) {
    const int r0 = (int)((int64_t)nR * g / nsplit), r1 = (int)((int64_t)nR * (g + 1) / nsplit);
    const int s0 = (int)sr.size();
    for (int r = r0; r < r1; ++r) {
      const auto& R = plan.R[r];
      const void* src = (R.kind == 0) ? (const void*)(Y + (size_t)R.idx * n * eb) : (const void*)(T + (size_t)R.idx * n * eb);
      sr.push_back({src, Rptr[r], chi_r, chi_r, chi_r, 0});
    }
    jr.push_back({(char*)partials + (size_t)g * n * eb, chi_r, Mr, chi_r, s0, (int)sr.size() - s0});
  }
  njobL = (int)jl.size();
  nopjob = (int)oj.size();
  njobR = (int)jr.size();
  // algorithmic work of the two contractions (formula terms) for profiling
  {
    const double d2 = (double)ds * dt;
    fl_L = 8.0 * d2 * chi_l * (double)chi_l * chi_r * wl;
    fl_R = 8.0 * d2 * chi_l * (double)chi_r * chi_r * wr;
    fl_all = (nsites == 2 && !raw_leg0) ? matvec_flops_formula(mpo, site, chi_l, chi_r) : fl_L + fl_R;
    const double ebs = (double)eb;
    // L: environments + theta in + Y out;  R: Y/T in + environments + partial out
    by_L = ebs * ((double)wl * chi_l * chi_l + (double)n + (double)plan.L.size() * n);
    by_R = ebs * ((double)plan.R.size() * n + (double)wr * chi_r * chi_r + (double)nsplit * n);
  }
  // one descriptor block
  size_t off = 0;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_jl = off; off = al(off + jl.size() * sizeof(GemmJob));
  const size_t o_sl = off; off = al(off + sl.size() * sizeof(GemmSeg));
  const size_t o_oj = off; off = al(off + std::max<size_t>(1, oj.size()) * sizeof(OpJob));
  const size_t o_ot = off; off = al(off + std::max<size_t>(1, ot.size()) * sizeof(OpTerm));
  const size_t o_jr = off; off = al(off + jr.size() * sizeof(GemmJob));
  const size_t o_sr = off; off = al(off + sr.size() * sizeof(GemmSeg));
  const size_t o_mj = off; off = al(off + std::max<size_t>(1, mixjobs.size() + mixjobsR.size()) * sizeof(MixJob));
  const size_t o_mt = off; off = al(off + std::max<size_t>(1, mixterms.size()) * sizeof(MixTerm));
  std::vector<char> host(off, 0);
  std::memcpy(host.data() + o_jl, jl.data(), jl.size() * sizeof(GemmJob));
  std::memcpy(host.data() + o_sl, sl.data(), sl.size() * sizeof(GemmSeg));
  std::memcpy(host.data() + o_oj, oj.data(), oj.size() * sizeof(OpJob));
  std::memcpy(host.data() + o_ot, ot.data(), ot.size() * sizeof(OpTerm));
  std::memcpy(host.data() + o_jr, jr.data(), jr.size() * sizeof(GemmJob));
  std::memcpy(host.data() + o_sr, sr.data(), sr.size() * sizeof(GemmSeg));
  std::vector<MixJob> allmix = mixjobs;
  allmix.insert(allmix.end(), mixjobsR.begin(), mixjobsR.end());
  std::memcpy(host.data() + o_mj, allmix.data(), allmix.size() * sizeof(MixJob));
  std::memcpy(host.data() + o_mt, mixterms.data(), mixterms.size() * sizeof(MixTerm));
  char* dd = (char*)ws_get(ctx, tag + ":desc", off);
  HIPCHK(hipMemcpyAsync(dd, host.data(), off, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));  // host staging buffer goes out of scope
  d_jobL = (GemmJob*)(dd + o_jl); d_segL = (GemmSeg*)(dd + o_sl);
  d_opjob = (OpJob*)(dd + o_oj); d_opterm = (OpTerm*)(dd + o_ot);
  d_jobR = (GemmJob*)(dd + o_jr); d_segR = (GemmSeg*)(dd + o_sr);
  // mixed environments (once per window)
  if (!mixjobs.empty())
    HIPCHK(launch_envmix(sprec, (MixJob*)(dd + o_mj), (int)mixjobs.size(), (MixTerm*)(dd + o_mt),
                         (int64_t)chi_l * chi_l, ctx->stream));
  if (!mixjobsR.empty())
    HIPCHK(launch_envmix(sprec, (MixJob*)(dd + o_mj) + mixjobs.size(), (int)mixjobsR.size(), (MixTerm*)(dd + o_mt),
                         (int64_t)chi_r * chi_r, ctx->stream));
}

void WindowOp::apply_left(const cf64* x) {
  const int sprec = (prec == PREC_FP64) ? PREC_FP64 : PREC_FP32;
  HIPCHK(launch_convert(sprec, xin, PREC_FP64, x, (int64_t)n, ctx->stream));
  HIPCHK(launch_cgemm(prec, 0, 0, d_jobL, njobL, d_segL, chi_l, ds * dt * chi_r, 0, ctx->stream));
}

void WindowOp::apply(const cf64* x, cf64* y) {
  hipStream_t st = ctx->stream;
  const int sprec = (prec == PREC_FP64) ? PREC_FP64 : PREC_FP32;
  tn_ctx::ProfSlot* ps = nullptr;
  if (ctx->prof) {
    ps = &ctx->pslot[ctx->pseq++ % tn_ctx::PROF_RING];
    if (ps->pending) prof_harvest(ctx, *ps);  // recorded PROF_RING matvecs ago: long complete
  }
  hipEvent_t* ev = ps ? ps->e : nullptr;
  if (ev) HIPCHK(hipEventRecord(ev[0], st));
  HIPCHK(launch_convert(sprec, xin, PREC_FP64, x, (int64_t)n, st));
  if (ev) HIPCHK(hipEventRecord(ev[1], st));
  HIPCHK(launch_cgemm(prec, 0, 0, d_jobL, njobL, d_segL, chi_l, ds * dt * chi_r, 0, st));
  if (ev) HIPCHK(hipEventRecord(ev[2], st));
  HIPCHK(launch_opapply(sprec, d_opjob, nopjob, d_opterm, chi_l, ds, dt, chi_r, st));
  if (ev) HIPCHK(hipEventRecord(ev[3], st));
  HIPCHK(launch_cgemm(prec, 0, 0, d_jobR, njobR, d_segR, chi_l * ds * dt, chi_r, 0, st));
  if (ev) HIPCHK(hipEventRecord(ev[4], st));
  HIPCHK(launch_reduce_partials(y, sprec, partials, nsplit, (int64_t)n, st));
  if (ps) {
    HIPCHK(hipEventRecord(ev[5], st));
    ps->fl[0] = fl_L;
    ps->fl[1] = fl_R;
    ps->fl[2] = fl_all;
    ps->by[0] = by_L;
    ps->by[1] = by_R;
    ps->pending = true;
  }
}

// ------------------------------------------------------------------ flop formulas
static void counts(const tn_mpo* mpo, int site, int& n_op, int& n_sc) {
  n_op = n_sc = 0;
  for (auto k : mpo->kinds[site]) {
    if ((k >= 2 && k <= 5) || (k >= 7 && k <= 9)) ++n_op;
    else if (k == 6) ++n_sc;
  }
}
double matvec_flops_formula(const tn_mpo* mpo, int s, int cl, int cr) {
  const double d = mpo->d;
  double f = 8.0 * d * d * cl * cr * ((double)mpo->w[s] * cl + (double)mpo->w[s + 2] * cr);
  for (int t = s; t <= s + 1; ++t) {
    int a, b;
    counts(mpo, t, a, b);
    f += 8.0 * d * d * d * cl * cr * a + 8.0 * d * d * cl * cr * b;
  }
  return f;
}
double env_flops_formula(const tn_mpo* mpo, int s, int cl, int cr) {
  const double d = mpo->d;
  int a, b;
  counts(mpo, s, a, b);
  return 8.0 * ((double)mpo->w[s] * cl * cl * d * cr + (double)a * d * d * cl * cr + (double)b * d * cl * cr +
                (double)mpo->w[s + 1] * cl * d * cr * cr);
}
