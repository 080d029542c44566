// Expectation values <psi|H|psi>/<psi|psi> of H = sum_t H_t with cached
// environments (Eq. 5, Sec. IV-B).
//
// Two boundary passes (top-down, bottom-up) store every intermediate boundary
// MPS.  A one-site or horizontal two-site term on row i is read from a
// three-layer strip (top environment of the rows above i, row i, bottom
// environment of the rows below); a vertical term on rows i, i+1 from a
// four-layer strip.  For every strip the left and right strip environments
// are contracted once (the right ones as left environments of the mirrored
// strip), then each site or bond yields a reduced density matrix by one more
// column transfer with the physical legs left open.  A term's value is
// tr(O rho) / tr(rho); the normalisation of the environments cancels.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "contract.h"
#include "peps.h"
#include "tape.h"

namespace hp {
namespace {

struct Ten {
  void* p = nullptr;
  std::string legs;
  std::vector<int64_t> dims;
  int64_t size() const {
    int64_t s = 1;
    for (auto d : dims) s *= d;
    return s;
  }
  TView view(bool conj = false) const { return tview_rm(p, legs, dims, conj); }
};

TView bview(const BndView& b, const std::string& legs) {
  return tview(b.p, legs, {b.n[0], b.n[1], b.n[2], b.n[3]}, {b.s[0], b.s[1], b.s[2], b.s[3]}, b.extent);
}
TView sview(const SiteView& s, const std::string& legs, bool conj) {
  return tview(s.p, legs, {s.n[0], s.n[1], s.n[2], s.n[3], s.n[4]}, {s.s[0], s.s[1], s.s[2], s.s[3], s.s[4]},
               s.extent, conj);
}

int64_t out_size(const TView& A, const TView& B, const std::string& out) {
  int64_t n = 1;
  for (char c : out) {
    const int64_t a = leg_dim(A, c), b = leg_dim(B, c);
    n *= a >= 0 ? a : b;
  }
  return n;
}

Ten contract(Ctx& ctx, bool cplx, const TView& A, const TView& B, const std::string& out) {
  Ten t;
  t.legs = out;
  const int64_t n = out_size(A, B, out);
  t.p = ctx.ws<double>(n * (cplx ? 2 : 1));
  t.dims = contract2(ctx, cplx, A, B, out, t.p, n);
  return t;
}

std::string spectators(const std::string& legs, const std::string& core) {
  std::string s;
  for (char c : legs)
    if (core.find(c) == std::string::npos) s += c;
  return s;
}

// the last contraction of a chain writes into a buffer allocated before the
// chain's scratch, so the scratch can be released
Ten alloc_out(Ctx& ctx, bool cplx, const TView& A, const TView& B, const std::string& out) {
  Ten t;
  t.legs = out;
  for (char c : out) {
    const int64_t a = leg_dim(A, c), b = leg_dim(B, c);
    t.dims.push_back(a >= 0 ? a : b);
  }
  t.p = ctx.ws<double>(t.size() * (cplx ? 2 : 1));
  return t;
}

// Number of chunks of the bottom-environment leg b (a spectator of every
// intermediate of a strip column until the last contraction sums it) that
// keeps each intermediate below the context's strip_chunk_bytes (1 GiB by
// default); 1 while a tape records (its adjoints need one product per
// output) or when everything fits.
int64_t strip_chunks(Ctx& ctx, bool cplx, const TView& L, const std::vector<TView>& ops,
                     const std::vector<std::string>& steps) {
  if (taping(ctx)) return 1;
  auto dim = [&](char c) {
    int64_t d = leg_dim(L, c);
    for (const auto& v : ops)
      if (d < 0) d = leg_dim(v, c);
    return d < 0 ? (int64_t)1 : d;
  };
  int64_t big = 0;
  for (const auto& st : steps) {
    int64_t n = 1;
    for (char c : st) n *= dim(c);
    big = std::max(big, n);
  }
  const int64_t bytes = big * (cplx ? 16 : 8);
  const int64_t budget = std::max<int64_t>(1, ctx.strip_chunk_bytes);
  return std::min(dim('b'), std::max<int64_t>(1, (bytes + budget - 1) / budget));
}

// One column of a three-layer strip: L[spec,t,l,L,b] -> L'[spec,s,r,R,c(,p,P)].
Ten transfer3(Ctx& ctx, bool cplx, const Ten& L, const BndView& top, const SiteView& ket, const SiteView& bra,
              const BndView& bot, bool open) {
  const std::string sp = spectators(L.legs, "tlLb");
  const std::string out = sp + (open ? "srRcpP" : "srRc");
  // output dims: spectators from L, s/c from the environments, r/R/p/P from the sites
  Ten res;
  res.legs = out;
  for (char ch : out) {
    int64_t dd = leg_dim(L.view(), ch);
    if (ch == 's') dd = top.n[3];
    if (ch == 'c') dd = bot.n[3];
    if (ch == 'r') dd = ket.n[3];
    if (ch == 'R') dd = bra.n[3];
    if (ch == 'p' || ch == 'P') dd = ket.n[4];
    res.dims.push_back(dd);
  }
  res.p = ctx.ws<double>(res.size() * (cplx ? 2 : 1));
  const std::string s1 = sp + "lLbuUs", s2 = sp + "LbUsdrp", s3 = sp + (open ? "bsdrDRpP" : "bsdrDR");
  const int64_t nch = strip_chunks(ctx, cplx, L.view(), {bview(top, "tuUs"), sview(ket, "udlrp", false),
                                                         sview(bra, "UDLRP", true), bview(bot, "bdDc")},
                                   {s1, s2, s3});
  const int64_t nbl = leg_dim(L.view(), 'b'), bc = (nbl + nch - 1) / nch;
  for (int64_t b0 = 0; b0 < nbl; b0 += bc) {
    const int64_t len = std::min(bc, nbl - b0);
    WsScope scope(ctx);
    Ten x1 = contract(ctx, cplx, restrict_leg(L.view(), 'b', b0, len, cplx), bview(top, "tuUs"), s1);
    Ten x2 = contract(ctx, cplx, x1.view(), sview(ket, "udlrp", false), s2);
    Ten x3 = contract(ctx, cplx, x2.view(), sview(bra, open ? "UDLRP" : "UDLRp", true), s3);
    contract2(ctx, cplx, x3.view(), restrict_leg(bview(bot, "bdDc"), 'b', b0, len, cplx), out, res.p, res.size(),
              b0 > 0);
  }
  return res;
}

// One column of a four-layer strip: L[spec,t,l,L,m,M,b] -> L'[spec,s,r,R,n,N,c(,p,P)(,q,Q)]: the
// upper row's physical legs stay open with open1, the lower row's with open2.
Ten transfer4(Ctx& ctx, bool cplx, const Ten& L, const BndView& top, const SiteView& k1, const SiteView& b1,
              const SiteView& k2, const SiteView& b2, const BndView& bot, bool open1, bool open2) {
  const std::string sp = spectators(L.legs, "tlLmMb");
  const std::string o1 = open1 ? "pP" : "", o2 = open2 ? "qQ" : "";
  const std::string out = sp + "srRnNc" + o1 + o2;
  Ten res;
  res.legs = out;
  for (char ch : out) {
    int64_t dd = leg_dim(L.view(), ch);
    if (ch == 's') dd = top.n[3];
    if (ch == 'c') dd = bot.n[3];
    if (ch == 'r') dd = k1.n[3];
    if (ch == 'R') dd = b1.n[3];
    if (ch == 'n') dd = k2.n[3];
    if (ch == 'N') dd = b2.n[3];
    if (ch == 'p' || ch == 'P' || ch == 'q' || ch == 'Q') dd = k1.n[4];
    res.dims.push_back(dd);
  }
  res.p = ctx.ws<double>(res.size() * (cplx ? 2 : 1));
  const std::string s1 = sp + "lLmMbuUs", s2 = sp + "LmMbUsvrp", s3 = sp + "mMbsvrVR" + o1,
                    s4 = sp + "MbsrVRdnq" + o1, s5 = sp + "bsrRdnDN" + o1 + o2;
  const int64_t nch = strip_chunks(ctx, cplx, L.view(), {bview(top, "tuUs"), sview(k1, "uvlrp", false),
                                                         sview(b1, "UVLRP", true), sview(k2, "vdmnq", false),
                                                         sview(b2, "VDMNQ", true), bview(bot, "bdDc")},
                                   {s1, s2, s3, s4, s5});
  const int64_t nbl = leg_dim(L.view(), 'b'), bc = (nbl + nch - 1) / nch;
  for (int64_t b0 = 0; b0 < nbl; b0 += bc) {
    const int64_t len = std::min(bc, nbl - b0);
    WsScope scope(ctx);
    Ten x1 = contract(ctx, cplx, restrict_leg(L.view(), 'b', b0, len, cplx), bview(top, "tuUs"), s1);
    Ten x2 = contract(ctx, cplx, x1.view(), sview(k1, "uvlrp", false), s2);
    Ten x3 = contract(ctx, cplx, x2.view(), sview(b1, open1 ? "UVLRP" : "UVLRp", true), s3);
    Ten x4 = contract(ctx, cplx, x3.view(), sview(k2, "vdmnq", false), s4);
    Ten x5 = contract(ctx, cplx, x4.view(), sview(b2, open2 ? "VDMNQ" : "VDMNq", true), s5);
    contract2(ctx, cplx, x5.view(), restrict_leg(bview(bot, "bdDc"), 'b', b0, len, cplx), out, res.p, res.size(),
              b0 > 0);
  }
  return res;
}

Ten ones(Ctx& ctx, bool cplx, const std::string& legs) {
  Ten t;
  t.legs = legs;
  t.dims.assign(legs.size(), 1);
  t.p = ctx.ws<double>(cplx ? 2 : 1);
  fill_value(ctx, (double*)t.p, 1, 1.0, cplx);
  return t;
}

// scalar terms: out[2t..2t+1] = tr(O rho) / tr(rho) (complex)
__global__ void expect_kernel(const double* const* rdm, const double* const* ops, const int* nsites, int d, int cplx,
                              int nterms, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nterms) return;
  const double* r = rdm[t];
  const double* o = ops[t];
  double nr = 0, ni = 0, dr = 0, di = 0;
  auto rho = [&](long long idx, double& re, double& im) {
    if (cplx) {
      re = r[2 * idx];
      im = r[2 * idx + 1];
    } else {
      re = r[idx];
      im = 0;
    }
  };
  if (nsites[t] == 1) {
    for (int p = 0; p < d; ++p)
      for (int P = 0; P < d; ++P) {
        double re, im;
        rho((long long)p * d + P, re, im);
        const double orr = o[2 * (P * d + p)], oi = o[2 * (P * d + p) + 1];
        nr += orr * re - oi * im;
        ni += orr * im + oi * re;
        if (p == P) {
          dr += re;
          di += im;
        }
      }
  } else {
    for (int p1 = 0; p1 < d; ++p1)
      for (int P1 = 0; P1 < d; ++P1)
        for (int p2 = 0; p2 < d; ++p2)
          for (int P2 = 0; P2 < d; ++P2) {
            double re, im;
            rho(((long long)(p1 * d + P1) * d + p2) * d + P2, re, im);
            const long long oo = ((P1 * d + P2) * d + p1) * d + p2;
            const double orr = o[2 * oo], oi = o[2 * oo + 1];
            nr += orr * re - oi * im;
            ni += orr * im + oi * re;
            if (p1 == P1 && p2 == P2) {
              dr += re;
              di += im;
            }
          }
  }
  const double den = dr * dr + di * di;
  out[2 * t] = (nr * dr + ni * di) / den;
  out[2 * t + 1] = (ni * dr - nr * di) / den;
}

// Cotangent of the reduced density matrices for the loss Re sum_t E_t,
// E_t = tr(O_t rho_t) / tr(rho_t): rhobar_t = conj(dE_t / drho_t) with
// dE / drho[e] = O-coefficient of rho[e] / tr(rho) - [e diagonal] E / tr(rho)
// (real lattices: the real part).  Terms that share a matrix accumulate one
// after the other (one workgroup, a barrier between terms).
__global__ void expect_bwd_kernel(const double* const* rdm, const double* const* ops, const int* nsites,
                                  const double* val, int d, int cplx, int nterms, double* const* grad) {
  for (int t = 0; t < nterms; ++t) {
    const double* r = rdm[t];
    const double* o = ops[t];
    double* g = grad[t];
    const int two = nsites[t] == 2;
    // tr(rho)
    double dr = 0, di = 0;
    const int nd = two ? d * d : d;
    for (int q = 0; q < nd; ++q) {
      long long idx;
      if (two) {
        const int p1 = q / d, p2 = q % d;
        idx = ((long long)(p1 * d + p1) * d + p2) * d + p2;
      } else {
        idx = (long long)q * d + q;
      }
      dr += cplx ? r[2 * idx] : r[idx];
      di += cplx ? r[2 * idx + 1] : 0.0;
    }
    const double den = dr * dr + di * di;
    const double er = val[2 * t], ei = val[2 * t + 1];
    const int nel = two ? d * d * d * d : d * d;
    for (int e = threadIdx.x; e < nel; e += blockDim.x) {
      long long oo;
      bool diag;
      if (two) {
        const int P2 = e % d, p2 = (e / d) % d, P1 = (e / (d * d)) % d, p1 = e / (d * d * d);
        oo = ((long long)(P1 * d + P2) * d + p1) * d + p2;
        diag = p1 == P1 && p2 == P2;
      } else {
        const int P = e % d, p = e / d;
        oo = (long long)P * d + p;
        diag = p == P;
      }
      double ar = o[2 * oo], ai = o[2 * oo + 1];
      if (diag) {
        ar -= er;
        ai -= ei;
      }
      // (ar + i ai) / (dr + i di)
      const double vr = (ar * dr + ai * di) / den, vi = (ai * dr - ar * di) / den;
      if (cplx) {
        g[2 * e] += vr;
        g[2 * e + 1] -= vi;
      } else {
        g[e] += vr;
      }
    }
    __syncthreads();
  }
}

}  // namespace
}  // namespace hp

namespace hp {

void check_terms(const Lattice& K, int n_terms, const int32_t* nsites, const int32_t* sites,
                 const int64_t* op_offset, bool diagonal) {
  const int nrow = K.nrow, ncol = K.ncol;
  for (int t = 0; t < n_terms; ++t) {
    const int* s = sites + 4 * t;
    HP_REQUIRE(nsites[t] == 1 || nsites[t] == 2, HPEPS_ERR_INVALID_ARG, "terms act on 1 or 2 sites");
    HP_REQUIRE(s[0] >= 0 && s[0] < nrow && s[1] >= 0 && s[1] < ncol, HPEPS_ERR_INVALID_ARG, "site out of range");
    if (nsites[t] == 2) {
      const bool horiz = s[2] == s[0] && s[3] == s[1] + 1, vert = s[3] == s[1] && s[2] == s[0] + 1;
      const bool diag = s[2] == s[0] + 1 && (s[3] == s[1] + 1 || s[3] == s[1] - 1) && s[3] >= 0 && s[3] < ncol;
      HP_REQUIRE(horiz || vert || (diagonal && diag), HPEPS_ERR_INVALID_ARG,
                 diagonal ? "two-site terms must be nearest or diagonal neighbours, site 1 first (above)"
                          : "two-site terms must be nearest neighbours, site 1 first");
    }
    HP_REQUIRE(op_offset[t] >= 0, HPEPS_ERR_INVALID_ARG, "bad operator offset");
  }
}

// Reduced density matrices rho_t (device, d^2 or d^4 elements, row-major
// [p, P] / [p1, P1, p2, P2]) of every term from the cached environments;
// terms on the same site or bond share one matrix.
std::vector<const double*> energy_rdms(Ctx& c, const Lattice& K, int n_terms, const int32_t* nsites,
                                       const int32_t* sites, const hpeps_esvd_opts& o) {
  const bool cplx = K.cplx;
  const int nrow = K.nrow, ncol = K.ncol, d = (int)K.sites[0].dims[4];
  double* logd = c.ws<double>(1);
  fill_value(c, logd, 1, 0.0, false);
  Lattice Kn = normalized_copy(c, K, logd);
  std::vector<std::vector<DevTensor>> tenv, benv;
  if (nrow > 1) {
    boundary_pass(c, Kn, Kn, kTop, o, nrow - 1, tenv, logd);
    boundary_pass(c, Kn, Kn, kBottom, o, nrow - 1, benv, logd);
  }
  // trivial environment
  const int es = cplx ? 2 : 1;
  std::vector<DevTensor> triv(ncol);
  for (auto& t : triv) {
    t.dims = {1, 1, 1, 1};
    t.p = c.ws<double>(es);
    fill_value(c, (double*)t.p, 1, 1.0, cplx);
  }
  auto top_of = [&](int i) -> const std::vector<DevTensor>& { return i == 0 ? triv : tenv[i - 1]; };
  auto bot_of = [&](int i) -> const std::vector<DevTensor>& { return i == nrow - 1 ? triv : benv[nrow - 2 - i]; };
  std::vector<const double*> rdm_ptr(n_terms, nullptr);
  // one reduced density matrix slot per term (d^4 elements), allocated
  // before the strips so that each strip's scratch can be released
  const int64_t slot = (int64_t)d * d * d * d * es;
  double* rdm_store = c.ws<double>(std::max<int64_t>(n_terms, 1) * slot);

  // a strip's inputs for the checkpoint: its environments and sites
  auto strip_inputs = [&](const std::vector<DevTensor>& top, const std::vector<DevTensor>& bot, int r0, int r1) {
    std::vector<std::pair<const void*, int64_t>> in;
    for (int j = 0; j < ncol; ++j) {
      in.push_back({top[j].p, top[j].size()});
      in.push_back({bot[j].p, bot[j].size()});
      for (int r = r0; r <= r1; ++r) in.push_back({Kn.at(r, j).p, Kn.at(r, j).size()});
    }
    return in;
  };

  // three-layer strips: one-site and horizontal terms (each strip one
  // checkpointed segment under a tape)
  for (int i = 0; i < nrow; ++i) {
    std::vector<int> here;
    for (int t = 0; t < n_terms; ++t)
      if (sites[4 * t] == i && (nsites[t] == 1 || sites[4 * t + 2] == i)) here.push_back(t);
    if (here.empty()) continue;
    // one reduced density matrix per (column, kind)
    std::vector<std::pair<int, int>> keys;
    std::vector<std::pair<void*, int64_t>> outs;
    for (int t : here) {
      const auto key = std::make_pair((int)sites[4 * t + 1], (int)nsites[t]);
      size_t k = 0;
      while (k < keys.size() && keys[k] != key) ++k;
      if (k == keys.size()) {
        keys.push_back(key);
        outs.push_back({rdm_store + (int64_t)t * slot, slot / es});
      }
      rdm_ptr[t] = (const double*)outs[k].first;
    }
    const std::vector<DevTensor> top = top_of(i), bot = bot_of(i);
    std::vector<DevTensor> row;
    for (int j = 0; j < ncol; ++j) row.push_back(Kn.at(i, j));
    auto run = [cplx, ncol, top, bot, row, keys, logd, slot, es](Ctx& c, const std::vector<void*>& dst) {
      WsScope strip_scope(c);
      auto col = [&](int j, Dir dir, BndView& tv, SiteView& kv, SiteView& bv, BndView& btv) {
        tv = orient_bnd(top[j], dir);
        kv = orient_site(row[j], kTop, dir);
        bv = kv;
        btv = orient_bnd(bot[j], dir);
      };
      std::vector<Ten> Lenv(ncol + 1), Renv(ncol + 1);
      Lenv[0] = ones(c, cplx, "tlLb");
      Renv[0] = ones(c, cplx, "tlLb");
      for (int q = 0; q < ncol; ++q) {
        BndView tv, btv;
        SiteView kv, bv;
        col(q, kL2R, tv, kv, bv, btv);
        Ten x = transfer3(c, cplx, Lenv[q], tv, kv, bv, btv, false);
        normalize(c, cplx, x.p, x.size(), 1, logd);
        x.legs = "tlLb";
        Lenv[q + 1] = x;
        col(ncol - 1 - q, kR2L, tv, kv, bv, btv);
        Ten y = transfer3(c, cplx, Renv[q], tv, kv, bv, btv, false);
        normalize(c, cplx, y.p, y.size(), 1, logd);
        y.legs = "tlLb";
        Renv[q + 1] = y;
      }
      for (size_t k = 0; k < keys.size(); ++k) {
        const int j = keys[k].first, kind = keys[k].second;
        BndView tv, btv;
        SiteView kv, bv;
        col(j, kL2R, tv, kv, bv, btv);
        Ten y = transfer3(c, cplx, Lenv[j], tv, kv, bv, btv, true);  // srRcpP
        if (kind == 1) {
          Ten R = Renv[ncol - 1 - j];
          R.legs = "srRc";
          contract2(c, cplx, y.view(), R.view(), "pP", dst[k], slot / es);
        } else {
          y.legs = "tlLbef";
          col(j + 1, kL2R, tv, kv, bv, btv);
          Ten y2 = transfer3(c, cplx, y, tv, kv, bv, btv, true);  // efsrRcpP
          Ten R = Renv[ncol - 2 - j];
          R.legs = "srRc";
          contract2(c, cplx, y2.view(), R.view(), "efpP", dst[k], slot / es);
        }
      }
    };
    run_segment(c, cplx, strip_inputs(top, bot, i, i), outs, run);
  }
  // four-layer strips: vertical and diagonal terms
  for (int i = 0; i + 1 < nrow; ++i) {
    std::vector<int> here;
    for (int t = 0; t < n_terms; ++t)
      if (nsites[t] == 2 && sites[4 * t] == i && sites[4 * t + 2] == i + 1) here.push_back(t);
    if (here.empty()) continue;
    // (column of site 1, column of site 2) -> rdm [p1,P1,p2,P2]
    std::vector<std::pair<int, int>> keys;
    std::vector<std::pair<void*, int64_t>> outs;
    for (int t : here) {
      const auto key = std::make_pair((int)sites[4 * t + 1], (int)sites[4 * t + 3]);
      size_t k = 0;
      while (k < keys.size() && keys[k] != key) ++k;
      if (k == keys.size()) {
        keys.push_back(key);
        outs.push_back({rdm_store + (int64_t)t * slot, slot / es});
      }
      rdm_ptr[t] = (const double*)outs[k].first;
    }
    const std::vector<DevTensor> top = top_of(i), bot = bot_of(i + 1);
    std::vector<DevTensor> r1, r2;
    for (int j = 0; j < ncol; ++j) {
      r1.push_back(Kn.at(i, j));
      r2.push_back(Kn.at(i + 1, j));
    }
    auto run = [cplx, ncol, top, bot, r1, r2, keys, logd, slot, es](Ctx& c, const std::vector<void*>& dst) {
      WsScope strip_scope(c);
      auto col = [&](int j, Dir dir, BndView& tv, SiteView& k1, SiteView& k2, BndView& btv) {
        tv = orient_bnd(top[j], dir);
        k1 = orient_site(r1[j], kTop, dir);
        k2 = orient_site(r2[j], kTop, dir);
        btv = orient_bnd(bot[j], dir);
      };
      std::vector<Ten> Lenv(ncol + 1), Renv(ncol + 1);
      Lenv[0] = ones(c, cplx, "tlLmMb");
      Renv[0] = ones(c, cplx, "tlLmMb");
      for (int q = 0; q < ncol; ++q) {
        BndView tv, btv;
        SiteView k1, k2;
        col(q, kL2R, tv, k1, k2, btv);
        Ten x = transfer4(c, cplx, Lenv[q], tv, k1, k1, k2, k2, btv, false, false);
        normalize(c, cplx, x.p, x.size(), 1, logd);
        x.legs = "tlLmMb";
        Lenv[q + 1] = x;
        col(ncol - 1 - q, kR2L, tv, k1, k2, btv);
        Ten y = transfer4(c, cplx, Renv[q], tv, k1, k1, k2, k2, btv, false, false);
        normalize(c, cplx, y.p, y.size(), 1, logd);
        y.legs = "tlLmMb";
        Renv[q + 1] = y;
      }
      for (size_t k = 0; k < keys.size(); ++k) {
        const int j = keys[k].first, j2 = keys[k].second;
        BndView tv, btv;
        SiteView k1, k2;
        if (j2 == j) {
          col(j, kL2R, tv, k1, k2, btv);
          Ten y = transfer4(c, cplx, Lenv[j], tv, k1, k1, k2, k2, btv, true, true);  // srRnNcpPqQ
          Ten R = Renv[ncol - 1 - j];
          R.legs = "srRnNc";
          contract2(c, cplx, y.view(), R.view(), "pPqQ", dst[k], slot / es);
        } else {
          // diagonal pair over columns a < a + 1: the first column opens the
          // site it holds, its open legs ride along as spectators (ef)
          const int a = std::min(j, j2);
          const bool first_upper = j < j2;  // down-right: the upper site is in column a
          col(a, kL2R, tv, k1, k2, btv);
          Ten y = transfer4(c, cplx, Lenv[a], tv, k1, k1, k2, k2, btv, first_upper, !first_upper);
          y.legs = "tlLmMbef";
          col(a + 1, kL2R, tv, k1, k2, btv);
          Ten y2 = transfer4(c, cplx, y, tv, k1, k1, k2, k2, btv, !first_upper, first_upper);
          Ten R = Renv[ncol - 2 - a];
          R.legs = "srRnNc";
          // y2 legs: ef (first column's open pair) + srRnNc + the second column's open pair
          contract2(c, cplx, y2.view(), R.view(), first_upper ? "efqQ" : "pPef", dst[k], slot / es);
        }
      }
    };
    run_segment(c, cplx, strip_inputs(top, bot, i, i + 1), outs, run);
  }
  return rdm_ptr;
}

// Term values tr(O rho) / tr(rho) on the device (2 doubles per term).
struct TermsDev {
  double* res = nullptr;
  const double* const* rp = nullptr;
  const double* const* op = nullptr;
  const int* ns = nullptr;
};

TermsDev term_values(Ctx& c, bool cplx, int d, int n_terms, const int32_t* nsites, const double* ops,
                     const int64_t* op_offset, const std::vector<const double*>& rdm_ptr) {
  TermsDev t;
  t.res = c.ws<double>(2 * std::max(n_terms, 1));
  if (n_terms == 0) return t;
  int64_t total = 0;
  for (int q = 0; q < n_terms; ++q)
    total = std::max<int64_t>(total, op_offset[q] + (nsites[q] == 1 ? d * d : d * d * d * d));
  double* ops_dev = c.ws<double>(2 * total);
  HP_CHECK_HIP(hipMemcpyAsync(ops_dev, ops, 2 * total * sizeof(double), hipMemcpyHostToDevice, c.stream));
  std::vector<const double*> op_ptr(n_terms);
  for (int q = 0; q < n_terms; ++q) op_ptr[q] = ops_dev + 2 * op_offset[q];
  auto* rp = c.ws<const double*>(n_terms);
  auto* op = c.ws<const double*>(n_terms);
  int* ns = c.ws<int>(n_terms);
  HP_CHECK_HIP(hipMemcpyAsync(rp, rdm_ptr.data(), n_terms * sizeof(void*), hipMemcpyHostToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(op, op_ptr.data(), n_terms * sizeof(void*), hipMemcpyHostToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(ns, nsites, n_terms * sizeof(int), hipMemcpyHostToDevice, c.stream));
  expect_kernel<<<cdiv(n_terms, 64), 64, 0, c.stream>>>(rp, op, ns, d, cplx ? 1 : 0, n_terms, t.res);
  HP_CHECK_HIP(hipGetLastError());
  t.rp = rp;
  t.op = op;
  t.ns = ns;
  return t;
}

// Synchronises; energy = sum of the term values, per_term optional.
void read_energy(Ctx& c, const TermsDev& t, int n_terms, double* energy, double* per_term) {
  std::vector<double> h(2 * std::max(n_terms, 1));
  HP_CHECK_HIP(hipMemcpyAsync(h.data(), t.res, h.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HP_CHECK_HIP(hipStreamSynchronize(c.stream));
  double er = 0, ei = 0;
  for (int q = 0; q < n_terms; ++q) {
    HP_REQUIRE(std::isfinite(h[2 * q]) && std::isfinite(h[2 * q + 1]), HPEPS_ERR_NUMERIC, "non-finite term value");
    er += h[2 * q];
    ei += h[2 * q + 1];
    if (per_term) {
      per_term[2 * q] = h[2 * q];
      per_term[2 * q + 1] = h[2 * q + 1];
    }
  }
  energy[0] = er;
  energy[1] = ei;
}

}  // namespace hp


// ---------------------------------------------------------------------------
// ABI

namespace {
template <class F>
hpeps_status guard_e(hpeps_ctx* ctx, F&& f) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  try {
    ctx->impl->ws_reset();
    f(*ctx->impl);
    return HPEPS_OK;
  } catch (const hp::Error& e) {
    ctx->impl->tape = nullptr;
    ctx->impl->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->impl->tape = nullptr;
    ctx->impl->last_error = "host allocation failed";
    return HPEPS_ERR_ALLOC;
  } catch (...) {
    ctx->impl->tape = nullptr;
    ctx->impl->last_error = "unknown error";
    return HPEPS_ERR_INVALID_ARG;
  }
}

void check_energy_args(const hpeps_esvd_opts* opts, int32_t n_terms, const int32_t* nsites, const int32_t* sites,
                       const double* ops, const int64_t* op_offset, const double* energy) {
  HP_REQUIRE(opts && opts->rank >= 1 && opts->oversample >= 0 && opts->power_iters >= 0, HPEPS_ERR_INVALID_ARG,
             "bad einsumsvd options");
  HP_REQUIRE(n_terms >= 0 && energy && (n_terms == 0 || (nsites && sites && ops && op_offset)),
             HPEPS_ERR_INVALID_ARG, "null argument");
}
}  // namespace

// ---------------------------------------------------------------------------
// Expectation values by whole contractions: Eq. 5 term by term without the
// cached environments, and the Trotter-Taylor estimate of Eq. 6.  Operators
// are applied exactly to the ket: a one-site operator on its site's physical
// leg; a two-site operator G[P,Q,p,q] (out1, out2, in1, in2) by the
// elementary split G = sum_{Q,q} G[:,Q,:,q] (x) |Q><q|: site 1 takes
// G[:,Q,:,q], site 2 takes |Q><q|, and (Q, q) is appended to their shared
// bond (index (b, Q, q) row-major, the bond grows from D to D d^2).  The bra
// (the original state) is zero-padded to the grown bonds, which does not
// change <psi|phi>.
namespace hp {
namespace {

__global__ void pad_kernel(const double* src, long long s0, long long s1, long long s2, long long s3,
                           long long s4, long long t1, long long t2, long long t3, long long t4, long long total,
                           int es, double* dst) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  long long r = e;
  const long long a4 = r % t4; r /= t4;
  const long long a3 = r % t3; r /= t3;
  const long long a2 = r % t2; r /= t2;
  const long long a1 = r % t1; r /= t1;
  const long long a0 = r;
  const bool in = a0 < s0 && a1 < s1 && a2 < s2 && a3 < s3 && a4 < s4;
  const long long si = in ? (((a0 * s1 + a1) * s2 + a2) * s3 + a3) * s4 + a4 : 0;
  for (int q = 0; q < es; ++q) dst[e * es + q] = in ? src[si * es + q] : 0.0;
}

// T zero-padded to dims (every leg at least as long as T's), in the workspace.
DevTensor pad_site(Ctx& c, bool cplx, const DevTensor& T, const std::vector<int64_t>& dims) {
  HP_REQUIRE(T.dims.size() == 5 && dims.size() == 5, HPEPS_ERR_SHAPE, "sites have five legs");
  for (int q = 0; q < 5; ++q) HP_REQUIRE(dims[q] >= T.dims[q], HPEPS_ERR_SHAPE, "padding cannot shrink a leg");
  DevTensor o;
  o.dims = dims;
  const long long total = o.size();
  o.p = c.ws<double>(total * (cplx ? 2 : 1));
  pad_kernel<<<cdiv(total, 256), 256, 0, c.stream>>>((const double*)T.p, T.dims[0], T.dims[1], T.dims[2],
                                                      T.dims[3], T.dims[4], dims[1], dims[2], dims[3], dims[4],
                                                      total, cplx ? 2 : 1, (double*)o.p);
  HP_CHECK_HIP(hipGetLastError());
  return o;
}

// A host operator (complex128 pairs, n entries) in the lattice's dtype on the
// device; a real lattice takes real operators only.
double* upload_op(Ctx& c, bool cplx, const double* op, int64_t n) {
  double* dev = c.ws<double>(n * (cplx ? 2 : 1));
  if (cplx) {
    HP_CHECK_HIP(hipMemcpyAsync(dev, op, 2 * n * sizeof(double), hipMemcpyHostToDevice, c.stream));
    return dev;
  }
  std::vector<double> re(n);
  for (int64_t i = 0; i < n; ++i) {
    HP_REQUIRE(op[2 * i + 1] == 0.0, HPEPS_ERR_DTYPE, "a complex operator needs a complex128 PEPS");
    re[i] = op[2 * i];
  }
  HP_CHECK_HIP(hipMemcpyAsync(dev, re.data(), n * sizeof(double), hipMemcpyHostToDevice, c.stream));
  HP_CHECK_HIP(hipStreamSynchronize(c.stream));  // re is released on return
  return dev;
}

DevTensor apply_one(Ctx& c, bool cplx, const DevTensor& T, const double* O, int d) {
  DevTensor o;
  o.dims = T.dims;
  o.p = c.ws<double>(o.size() * (cplx ? 2 : 1));
  contract2(c, cplx, tview_rm(T.p, "udlrp", T.dims), tview_rm(O, "Pp", {d, d}), "udlrP", o.p, o.size());
  return o;
}

// Exact two-site application (elementary split); E[w,Q,q,X] =
// delta(w, q) delta(Q, X) (the d^2 x d^2 identity), so that site 2 becomes
// sum_w T[.., w] E[w,Q,q,X] = delta(Q, X) T[.., q].
void apply_two(Ctx& c, bool cplx, DevTensor& S, DevTensor& T, bool vertical, const double* G, const double* E,
               int d) {
  const TView g = tview_rm(G, "PQpq", {d, d, d, d});
  const TView e = tview_rm(E, "wQqX", {d, d, d, d});
  const int64_t dd = (int64_t)d * d;
  DevTensor S2, T2;
  if (vertical) {
    S2.dims = {S.dims[0], S.dims[1] * dd, S.dims[2], S.dims[3], d};
    T2.dims = {T.dims[0] * dd, T.dims[1], T.dims[2], T.dims[3], d};
  } else {
    S2.dims = {S.dims[0], S.dims[1], S.dims[2], S.dims[3] * dd, d};
    T2.dims = {T.dims[0], T.dims[1], T.dims[2] * dd, T.dims[3], d};
  }
  S2.p = c.ws<double>(S2.size() * (cplx ? 2 : 1));
  T2.p = c.ws<double>(T2.size() * (cplx ? 2 : 1));
  contract2(c, cplx, tview_rm(S.p, "udlrp", S.dims), g, vertical ? "udQqlrP" : "udlrQqP", S2.p, S2.size());
  contract2(c, cplx, tview_rm(T.p, "udlrw", T.dims), e, vertical ? "uQqdlrX" : "udlQqrX", T2.p, T2.size());
  S = S2;
  T = T2;
}

// <psi|phi> / <psi|psi> from two norm results (log, phase re, im).
void ratio_of(const double* num, const double* den, double* out) {
  const double m = std::exp(num[0] - den[0]);
  // (a / b) with unit-modulus b: a * conj(b)
  out[0] = m * (num[1] * den[1] + num[2] * den[2]);
  out[1] = m * (num[2] * den[1] - num[1] * den[2]);
}

void read3(Ctx& c, const double* dev, double* h) {
  HP_CHECK_HIP(hipMemcpyAsync(h, dev, 3 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HP_CHECK_HIP(hipStreamSynchronize(c.stream));
  HP_REQUIRE(std::isfinite(h[0]) && std::isfinite(h[1]) && std::isfinite(h[2]), HPEPS_ERR_NUMERIC,
             "non-finite overlap");
}

}  // namespace
}  // namespace hp

extern "C" hpeps_status hpeps_peps_energy_uncached(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_terms,
                                                   const int32_t* nsites, const int32_t* sites, const double* ops,
                                                   const int64_t* op_offset, const hpeps_esvd_opts* opts,
                                                   double* energy, double* per_term) {
  using namespace hp;
  return guard_e(ctx, [&](Ctx& c) {
    check_energy_args(opts, n_terms, nsites, sites, ops, op_offset, energy);
    const Lattice K = lattice_from_abi(ket);
    check_terms(K, n_terms, nsites, sites, op_offset, false);
    const bool cplx = K.cplx;
    const int d = (int)K.sites[0].dims[4];
    double* dev = c.ws<double>(3);
    norm_lattices(c, K, K, *opts, dev);
    double h0[3];
    read3(c, dev, h0);
    double* E = c.ws<double>((int64_t)d * d * d * d * (cplx ? 2 : 1));
    fill_identity(c, E, (int64_t)d * d, 1, cplx);
    double er = 0, ei = 0;
    for (int t = 0; t < n_terms; ++t) {
      WsScope scope(c);
      const int* s = sites + 4 * t;
      Lattice phi = K, bra = K;
      const size_t a = (size_t)s[0] * K.ncol + s[1];
      if (nsites[t] == 1) {
        phi.sites[a] = apply_one(c, cplx, K.sites[a], upload_op(c, cplx, ops + 2 * op_offset[t], (int64_t)d * d), d);
      } else {
        const size_t b = (size_t)s[2] * K.ncol + s[3];
        apply_two(c, cplx, phi.sites[a], phi.sites[b], s[2] == s[0] + 1,
                  upload_op(c, cplx, ops + 2 * op_offset[t], (int64_t)d * d * d * d), E, d);
        bra.sites[a] = pad_site(c, cplx, K.sites[a], phi.sites[a].dims);
        bra.sites[b] = pad_site(c, cplx, K.sites[b], phi.sites[b].dims);
      }
      double* dv = c.ws<double>(3);
      norm_lattices(c, phi, bra, *opts, dv);
      double h[3], v[2];
      read3(c, dv, h);
      ratio_of(h, h0, v);
      er += v[0];
      ei += v[1];
      if (per_term) {
        per_term[2 * t] = v[0];
        per_term[2 * t + 1] = v[1];
      }
    }
    energy[0] = er;
    energy[1] = ei;
  });
}

extern "C" hpeps_status hpeps_peps_trotter_expectation(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_gates,
                                                       const int32_t* sites, const double* gates, double tau,
                                                       const hpeps_esvd_opts* opts, double* estimate,
                                                       double* ratio) {
  using namespace hp;
  return guard_e(ctx, [&](Ctx& c) {
    HP_REQUIRE(opts && opts->rank >= 1 && opts->oversample >= 0 && opts->power_iters >= 0, HPEPS_ERR_INVALID_ARG,
               "bad einsumsvd options");
    HP_REQUIRE(n_gates >= 1 && sites && gates && estimate, HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(tau != 0.0 && std::isfinite(tau), HPEPS_ERR_INVALID_ARG, "tau must be finite and nonzero");
    const Lattice K = lattice_from_abi(ket);
    const bool cplx = K.cplx;
    const int d = (int)K.sites[0].dims[4];
    const int64_t g4 = (int64_t)d * d * d * d;
    std::vector<int32_t> two(n_gates, 2);
    std::vector<int64_t> off(n_gates);
    for (int t = 0; t < n_gates; ++t) off[t] = t * g4;
    check_terms(K, n_gates, two.data(), sites, off.data(), false);
    double* E = c.ws<double>((int64_t)d * d * d * d * (cplx ? 2 : 1));
    fill_identity(c, E, (int64_t)d * d, 1, cplx);
    // phi = prod_j G_j psi, gates in the order given
    Lattice phi = K;
    for (int t = 0; t < n_gates; ++t) {
      const int* s = sites + 4 * t;
      apply_two(c, cplx, phi.sites[(size_t)s[0] * K.ncol + s[1]], phi.sites[(size_t)s[2] * K.ncol + s[3]],
                s[2] == s[0] + 1, upload_op(c, cplx, gates + 2 * off[t], g4), E, d);
    }
    Lattice bra = K;
    for (size_t q = 0; q < K.sites.size(); ++q) bra.sites[q] = pad_site(c, cplx, K.sites[q], phi.sites[q].dims);
    double* dv = c.ws<double>(6);
    norm_lattices(c, phi, bra, *opts, dv);
    norm_lattices(c, K, K, *opts, dv + 3);
    double h1[3], h0[3], r[2];
    read3(c, dv, h1);
    read3(c, dv + 3, h0);
    ratio_of(h1, h0, r);
    estimate[0] = (r[0] - 1.0) / tau;
    estimate[1] = r[1] / tau;
    if (ratio) {
      ratio[0] = r[0];
      ratio[1] = r[1];
    }
  });
}

extern "C" hpeps_status hpeps_peps_energy(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_terms,
                                          const int32_t* nsites, const int32_t* sites, const double* ops,
                                          const int64_t* op_offset, const hpeps_esvd_opts* opts, double* energy,
                                          double* per_term) {
  using namespace hp;
  return guard_e(ctx, [&](Ctx& c) {
    check_energy_args(opts, n_terms, nsites, sites, ops, op_offset, energy);
    Lattice K = lattice_from_abi(ket);
    check_terms(K, n_terms, nsites, sites, op_offset, true);
    const auto rdm = energy_rdms(c, K, n_terms, nsites, sites, *opts);
    const TermsDev t = term_values(c, K.cplx, (int)K.sites[0].dims[4], n_terms, nsites, ops, op_offset, rdm);
    read_energy(c, t, n_terms, energy, per_term);
  });
}

extern "C" hpeps_status hpeps_peps_energy_backward(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_terms,
                                                   const int32_t* nsites, const int32_t* sites, const double* ops,
                                                   const int64_t* op_offset, const hpeps_esvd_opts* opts,
                                                   double broadening, void* const* grads, double* energy) {
  using namespace hp;
  return guard_e(ctx, [&](Ctx& c) {
    check_energy_args(opts, n_terms, nsites, sites, ops, op_offset, energy);
    HP_REQUIRE(grads, HPEPS_ERR_INVALID_ARG, "null gradient array");
    HP_REQUIRE(broadening >= 0.0, HPEPS_ERR_INVALID_ARG, "broadening must be >= 0");
    Lattice K = lattice_from_abi(ket);
    check_terms(K, n_terms, nsites, sites, op_offset, false);
    for (size_t q = 0; q < K.sites.size(); ++q) HP_REQUIRE(grads[q], HPEPS_ERR_INVALID_ARG, "null gradient pointer");
    const int d = (int)K.sites[0].dims[4];
    Tape tape(K.cplx);
    for (auto& s : K.sites) tape.mark_input(s.p, s.size());
    c.tape = &tape;
    const auto rdm = energy_rdms(c, K, n_terms, nsites, sites, *opts);
    c.tape = nullptr;
    const TermsDev t = term_values(c, K.cplx, d, n_terms, nsites, ops, op_offset, rdm);
    if (n_terms > 0) {
      std::vector<double*> gr(n_terms);
      for (int q = 0; q < n_terms; ++q) gr[q] = tape.grad(c, rdm[q]);
      auto* gp = c.ws<double*>(n_terms);
      HP_CHECK_HIP(hipMemcpyAsync(gp, gr.data(), n_terms * sizeof(void*), hipMemcpyHostToDevice, c.stream));
      expect_bwd_kernel<<<1, 256, 0, c.stream>>>(t.rp, t.op, t.ns, t.res, d, K.cplx ? 1 : 0, n_terms, gp);
      HP_CHECK_HIP(hipGetLastError());
    }
    tape.backward(c, broadening);
    write_site_grads(c, tape, K, grads);
    read_energy(c, t, n_terms, energy, nullptr);
  });
}
