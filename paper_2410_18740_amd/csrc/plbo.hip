// Gate-parameterised local basis (Sec. III.B).
//
// The basis of a mode is U|m>, m < d, with
//   U = D(alpha) S(r e^{i phi}) R(theta) P2(s) P3(gamma) K(kappa),
//   p = (alpha_x, alpha_p, r, phi, theta, s, gamma, kappa),
// so its operators are the blocks <m|U^dag O U|n>.  U^dag a U has the closed
// form of eq. SymplecticBasisTransformation: a polynomial of degree two in a
// and a^dag with photon-number phases from the Kerr gate.  It is assembled at
// d + 4 levels, where every entry of the d x d block of a product of two
// quadratures is exact, and truncated to d (SM Sec. 5).  All matrices are
// banded (U^dag a U reaches two levels up and down), so products cost
// O(d) per band entry.  Derivatives in the eight parameters are carried
// forward alongside the values (forward-mode differentiation).
//
// On the device: the slot environments G_k[n'][n] = dE/dO_k[n'][n] of a
// single-site window (the energy is linear in each site operator), reduced
// from the left-contracted tensors Y = L x and the right-contracted
// conjugates U = x R^H of the window operator.
//
// The Fock image U[:D, :d] for photon-number observables applies the six
// gates to the first d Fock states in a larger space, each as exp(G) v by a
// truncated Taylor series over sub-steps with |G| / steps <= 1 (the scaling
// idea of Al-Mohy and Higham's expmv); the generators are banded.
#include <algorithm>
#include <cmath>
#include <cstring>
#include "internal.h"

namespace {
constexpr int NP = TN_PLBO_NPARAM;

// value and gradient in the eight parameters
struct Dc {
  cd v = 0.0;
  cd g[NP] = {};
};
Dc dconst(cd v) {
  Dc r;
  r.v = v;
  return r;
}
Dc dparam(int j, double v) {
  Dc r;
  r.v = v;
  r.g[j] = 1.0;
  return r;
}
Dc operator+(const Dc& a, const Dc& b) {
  Dc r;
  r.v = a.v + b.v;
  for (int j = 0; j < NP; ++j) r.g[j] = a.g[j] + b.g[j];
  return r;
}
Dc operator-(const Dc& a, const Dc& b) {
  Dc r;
  r.v = a.v - b.v;
  for (int j = 0; j < NP; ++j) r.g[j] = a.g[j] - b.g[j];
  return r;
}
Dc operator*(const Dc& a, const Dc& b) {
  Dc r;
  r.v = a.v * b.v;
  for (int j = 0; j < NP; ++j) r.g[j] = a.g[j] * b.v + a.v * b.g[j];
  return r;
}
Dc operator*(cd s, const Dc& a) {
  Dc r;
  r.v = s * a.v;
  for (int j = 0; j < NP; ++j) r.g[j] = s * a.g[j];
  return r;
}
// e^{i x} for a real-valued x
Dc dexpi(const Dc& x) {
  const cd e = std::exp(cd(0.0, x.v.real()));
  Dc r;
  r.v = e;
  for (int j = 0; j < NP; ++j) r.g[j] = cd(0.0, 1.0) * e * x.g[j];
  return r;
}
Dc dcosh(const Dc& x) {
  Dc r;
  r.v = std::cosh(x.v.real());
  for (int j = 0; j < NP; ++j) r.g[j] = std::sinh(x.v.real()) * x.g[j];
  return r;
}
Dc dsinh(const Dc& x) {
  Dc r;
  r.v = std::sinh(x.v.real());
  for (int j = 0; j < NP; ++j) r.g[j] = std::cosh(x.v.real()) * x.g[j];
  return r;
}

// dense n x n storage with a stated half bandwidth; value and gradients
struct BMat {
  int n = 0, bw = 0;
  std::vector<Dc> e;
  BMat(int n_, int bw_) : n(n_), bw(bw_), e((size_t)n_ * n_) {}
  Dc& at(int i, int j) { return e[(size_t)i * n + j]; }
  const Dc& at(int i, int j) const { return e[(size_t)i * n + j]; }
};
BMat adjoint(const BMat& A) {
  BMat R(A.n, A.bw);
  for (int i = 0; i < A.n; ++i)
    for (int j = std::max(0, i - A.bw); j <= std::min(A.n - 1, i + A.bw); ++j) {
      const Dc& s = A.at(j, i);
      Dc& t = R.at(i, j);
      t.v = std::conj(s.v);
      for (int k = 0; k < NP; ++k) t.g[k] = std::conj(s.g[k]);
    }
  return R;
}
BMat lincomb(cd a, const BMat& A, cd b, const BMat& B) {
  BMat R(A.n, std::max(A.bw, B.bw));
  for (size_t i = 0; i < R.e.size(); ++i) R.e[i] = a * A.e[i] + b * B.e[i];
  return R;
}
BMat matmul(const BMat& A, const BMat& B) {
  const int n = A.n;
  BMat R(n, A.bw + B.bw);
  for (int i = 0; i < n; ++i)
    for (int k = std::max(0, i - A.bw); k <= std::min(n - 1, i + A.bw); ++k) {
      const Dc& a = A.at(i, k);
      for (int j = std::max(0, k - B.bw); j <= std::min(n - 1, k + B.bw); ++j) {
        const Dc& b = B.at(k, j);
        Dc& r = R.at(i, j);
        r.v += a.v * b.v;
        for (int q = 0; q < NP; ++q) r.g[q] += a.g[q] * b.v + a.v * b.g[q];
      }
    }
  return R;
}

// U^dag a U at n levels (eq. SymplecticBasisTransformation)
BMat transformed_a(int n, const double* p) {
  const cd I(0.0, 1.0);
  const Dc ax = dparam(0, p[0]), ap = dparam(1, p[1]), r = dparam(2, p[2]), phi = dparam(3, p[3]),
           th = dparam(4, p[4]), s = dparam(5, p[5]), g = dparam(6, p[6]), k = dparam(7, p[7]);
  const Dc e1 = dexpi(th), e2 = dexpi(phi - th), ch = dcosh(r), sh = dsinh(r);
  const Dc is2 = (0.5 * I) * s;
  const Dc one = dconst(1.0);
  const Dc c1 = (one + is2) * e1 * ch + is2 * e2 * sh;
  const Dc c2 = (one - is2) * e2 * sh - is2 * e1 * ch;
  const Dc c3 = e1 * ch + e2 * sh;
  const Dc cub = (0.5 * I) * g * c3;
  const Dc al = ax + I * ap;
  BMat A(n, 2);
  for (int m = 0; m < n; ++m) {
    A.at(m, m) = cub * dconst(2.0 * m + 1.0) + al;
    if (m + 1 < n) {  // a e^{i kappa (2 n - 1)}: <m|a|m+1> sqrt(m+1), phase at n = m + 1
      const int q = m + 1;
      A.at(m, q) = c1 * dexpi((double)(2 * q - 1) * k) * dconst(std::sqrt((double)q));
    }
    if (m >= 1) {  // e^{-i kappa (2 n - 1)} a^dag: phase at n = m
      A.at(m, m - 1) = dconst(-1.0) * c2 * dexpi((double)(-(2 * m - 1)) * k) * dconst(std::sqrt((double)m));
    }
    if (m + 2 < n) {  // a a e^{i 4 kappa (n - 1)}: phase at n = m + 2
      const int q = m + 2;
      A.at(m, q) = cub * dexpi((double)(4 * (q - 1)) * k) * dconst(std::sqrt((double)q * (q - 1)));
    }
    if (m >= 2) {  // e^{-i 4 kappa (n - 1)} a^dag a^dag: phase at n = m
      A.at(m, m - 2) = cub * dexpi((double)(-4 * (m - 1)) * k) * dconst(std::sqrt((double)m * (m - 1)));
    }
  }
  return A;
}
}  // namespace

void plbo_local_ops(int d, const double* p, double a_ss, double b_ss, double g_ss, std::vector<cd>& ops,
                    std::vector<cd>* dops) {
  const int n = d + 4;
  const BMat A = transformed_a(n, p);
  const BMat Ah = adjoint(A);
  const double r2 = 1.0 / std::sqrt(2.0);
  const cd I(0.0, 1.0);
  const BMat X = lincomb(r2, A, r2, Ah);
  const BMat P = lincomb(-I * r2, A, I * r2, Ah);
  const BMat X2 = matmul(X, X), P2 = matmul(P, P);
  const BMat Pt = lincomb(1.0, matmul(X, P), 1.0, matmul(P, X));
  const size_t dd = (size_t)d * d;
  ops.assign((size_t)NOPS * dd, 0.0);
  if (dops) dops->assign((size_t)NP * NOPS * dd, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const Dc* src[4] = {&X.at(i, j), &P.at(i, j), &X2.at(i, j), &Pt.at(i, j)};
      const Dc& pp = P2.at(i, j);
      Dc S = (0.5 * a_ss) * *src[2] + (0.5 * b_ss) * pp + (0.5 * g_ss) * *src[3];
      if (i == j) S.v -= 0.5;
      const Dc* slot[NOPS] = {src[0], src[1], &S, src[2], src[3]};
      for (int o = 0; o < NOPS; ++o) {
        ops[(size_t)o * dd + (size_t)i * d + j] = slot[o]->v;
        if (dops)
          for (int q = 0; q < NP; ++q) (*dops)[((size_t)q * NOPS + o) * dd + (size_t)i * d + j] = slot[o]->g[q];
      }
    }
}

// ------------------------------------------------------------------ site functional and optimisers
// W^dag O W for each d_big x d_big block of `in` (count blocks) -> d x d blocks
static void project_blocks(const std::vector<cd>& in, int count, int D, const std::vector<cd>& W, int d,
                           std::vector<cd>& out) {
  out.assign((size_t)count * d * d, 0.0);
  std::vector<cd> t((size_t)D * d);
  for (int c = 0; c < count; ++c) {
    const cd* O = in.data() + (size_t)c * D * D;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < d; ++j) {
        cd a = 0.0;
        for (int k = 0; k < D; ++k) a += O[(size_t)i * D + k] * W[(size_t)k * d + j];
        t[(size_t)i * d + j] = a;
      }
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        cd a = 0.0;
        for (int k = 0; k < D; ++k) a += std::conj(W[(size_t)k * d + i]) * t[(size_t)k * d + j];
        out[((size_t)c * d + i) * d + j] = a;
      }
  }
}

double plbo_site_energy(const PlboSite& S, const double* p, double* grad) {
  const int d = S.d;
  const size_t dd = (size_t)d * d;
  const std::vector<cd>& G = *S.G;
  std::vector<cd> ops, dops;
  if (S.W) {
    std::vector<cd> big, dbig;
    plbo_local_ops(S.D, p, S.a_ss, S.b_ss, S.g_ss, big, grad ? &dbig : nullptr);
    project_blocks(big, NOPS, S.D, *S.W, d, ops);
    if (grad) project_blocks(dbig, NP * NOPS, S.D, *S.W, d, dops);
  } else {
    plbo_local_ops(d, p, S.a_ss, S.b_ss, S.g_ss, ops, grad ? &dops : nullptr);
  }
  double e = 0.0;
  for (int i = 0; i < d; ++i) e += G[(size_t)i * d + i].real();
  for (int k = 1; k <= NOPS; ++k)
    for (size_t q = 0; q < dd; ++q) e += (G[k * dd + q] * ops[(k - 1) * dd + q]).real();
  if (grad)
    for (int j = 0; j < NP; ++j) {
      double g = 0.0;
      for (int k = 1; k <= NOPS; ++k)
        for (size_t q = 0; q < dd; ++q) g += (G[k * dd + q] * dops[((size_t)j * NOPS + k - 1) * dd + q]).real();
      grad[j] = g;
    }
  return e;
}

// Adam (Kingma & Ba): moments m, v and step count t carried by the caller.
// L-BFGS (Nocedal, Math. Comp. 35, 1980: two-loop recursion over the last
// eight curvature pairs, started afresh on every call) with a backtracking
// Armijo line search on the exact site energy; a pair whose curvature
// s^T y is not positive is skipped.  Both move only the masked parameters.
void plbo_optimise(const PlboSite& S, const tn_plbo_opts& po, double* p, double* m, double* v, int* t) {
  auto masked = [&](double* g) {
    for (int j = 0; j < NP; ++j)
      if (!((po.mask >> j) & 1u)) g[j] = 0.0;
  };
  double g[NP];
  if (po.optimizer == TN_PLBO_ADAM) {
    for (int it = 0; it < po.steps; ++it) {
      plbo_site_energy(S, p, g);
      masked(g);
      const int tt = ++*t;
      const double c1 = 1.0 - std::pow(po.beta1, tt), c2 = 1.0 - std::pow(po.beta2, tt);
      for (int j = 0; j < NP; ++j) {
        if (!((po.mask >> j) & 1u)) continue;
        m[j] = po.beta1 * m[j] + (1.0 - po.beta1) * g[j];
        v[j] = po.beta2 * v[j] + (1.0 - po.beta2) * g[j] * g[j];
        p[j] -= po.lr * (m[j] / c1) / (std::sqrt(v[j] / c2) + po.eps);
      }
    }
    return;
  }
  constexpr int HIST = 8;
  std::vector<std::array<double, NP>> sk, yk;
  std::vector<double> rho;
  double f = plbo_site_energy(S, p, g);
  masked(g);
  for (int it = 0; it < po.steps; ++it) {
    double gmax = 0.0;
    for (int j = 0; j < NP; ++j) gmax = std::max(gmax, std::fabs(g[j]));
    if (!(gmax > 0.0)) break;
    // two-loop recursion: d = -H g
    double q[NP], al[HIST];
    for (int j = 0; j < NP; ++j) q[j] = g[j];
    for (int h = (int)sk.size() - 1; h >= 0; --h) {
      double a = 0.0;
      for (int j = 0; j < NP; ++j) a += sk[h][j] * q[j];
      a *= rho[h];
      al[h] = a;
      for (int j = 0; j < NP; ++j) q[j] -= a * yk[h][j];
    }
    double gam = 1.0;
    if (!sk.empty()) {
      double sy = 0.0, yy = 0.0;
      for (int j = 0; j < NP; ++j) {
        sy += sk.back()[j] * yk.back()[j];
        yy += yk.back()[j] * yk.back()[j];
      }
      gam = sy / yy;
    } else {
      gam = po.lr / gmax;  // first step: at most lr in any parameter
    }
    for (int j = 0; j < NP; ++j) q[j] *= gam;
    for (size_t h = 0; h < sk.size(); ++h) {
      double b = 0.0;
      for (int j = 0; j < NP; ++j) b += yk[h][j] * q[j];
      b *= rho[h];
      for (int j = 0; j < NP; ++j) q[j] += sk[h][j] * (al[h] - b);
    }
    double dir[NP], slope = 0.0;
    for (int j = 0; j < NP; ++j) {
      dir[j] = -q[j];
      slope += dir[j] * g[j];
    }
    if (!(slope < 0.0)) {  // not a descent direction: restart from the scaled gradient
      sk.clear();
      yk.clear();
      rho.clear();
      for (int j = 0; j < NP; ++j) dir[j] = -(po.lr / gmax) * g[j];
      slope = 0.0;
      for (int j = 0; j < NP; ++j) slope += dir[j] * g[j];
    }
    double step = 1.0, pn[NP], gn[NP], fn = f;
    bool ok = false;
    for (int ls = 0; ls < 40; ++ls) {
      for (int j = 0; j < NP; ++j) pn[j] = p[j] + step * dir[j];
      fn = plbo_site_energy(S, pn, gn);
      if (std::isfinite(fn) && fn <= f + 1e-4 * step * slope) {
        ok = true;
        break;
      }
      step *= 0.5;
    }
    if (!ok) break;
    masked(gn);
    std::array<double, NP> s1{}, y1{};
    double sy = 0.0;
    for (int j = 0; j < NP; ++j) {
      s1[j] = pn[j] - p[j];
      y1[j] = gn[j] - g[j];
      sy += s1[j] * y1[j];
    }
    if (sy > 1e-300) {
      if ((int)sk.size() == HIST) {
        sk.erase(sk.begin());
        yk.erase(yk.begin());
        rho.erase(rho.begin());
      }
      sk.push_back(s1);
      yk.push_back(y1);
      rho.push_back(1.0 / sy);
    }
    for (int j = 0; j < NP; ++j) {
      p[j] = pn[j];
      g[j] = gn[j];
    }
    f = fn;
  }
}

// ------------------------------------------------------------------ Fock image of the basis
namespace {
// y = G x for a banded generator stored by diagonals: G[i][i+o] = diag[o + 3][i]
struct Banded {
  int n;
  std::vector<cd> dg[7];  // offsets -3..3
  explicit Banded(int n_) : n(n_) {
    for (auto& v : dg) v.assign(n_, 0.0);
  }
  void apply(const std::vector<cd>& x, std::vector<cd>& y) const {
    for (int i = 0; i < n; ++i) {
      cd s = 0.0;
      for (int o = -3; o <= 3; ++o) {
        const int j = i + o;
        if (j >= 0 && j < n) s += dg[o + 3][i] * x[j];
      }
      y[i] = s;
    }
  }
  double norm1() const {  // max column sum of |G|
    double m = 0.0;
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int o = -3; o <= 3; ++o) {
        const int i = j - o;
        if (i >= 0 && i < n) s += std::abs(dg[o + 3][i]);
      }
      m = std::max(m, s);
    }
    return m;
  }
};
// x <- exp(G) x: steps sub-steps of a Taylor series truncated when a term is
// below 1e-18 of the partial sum
void expmv(const Banded& G, std::vector<cd>& x) {
  const double nrm = G.norm1();
  const int steps = std::max(1, (int)std::ceil(nrm));
  const double h = 1.0 / steps;
  std::vector<cd> term(x.size()), nxt(x.size()), acc(x.size());
  for (int st = 0; st < steps; ++st) {
    acc = x;
    term = x;
    for (int k = 1; k < 200; ++k) {
      G.apply(term, nxt);
      double tn = 0.0, an = 0.0;
      for (size_t i = 0; i < x.size(); ++i) {
        term[i] = nxt[i] * (h / k);
        acc[i] += term[i];
        tn = std::max(tn, std::abs(term[i]));
        an = std::max(an, std::abs(acc[i]));
      }
      if (tn <= 1e-18 * an) break;
    }
    x = acc;
  }
}
// (a + a^dag)^k entries on offsets, exact block of the infinite operator
Banded quad_poly(int n, int power, cd coef) {
  // build the dense block at n + power levels and read the band
  const int m = n + power;
  std::vector<double> y((size_t)m * m, 0.0), t((size_t)m * m, 0.0), acc((size_t)m * m, 0.0);
  for (int i = 0; i + 1 < m; ++i) y[(size_t)i * m + i + 1] = y[(size_t)(i + 1) * m + i] = std::sqrt((double)(i + 1));
  for (int i = 0; i < m; ++i) acc[(size_t)i * m + i] = 1.0;
  for (int q = 0; q < power; ++q) {
    std::fill(t.begin(), t.end(), 0.0);
    for (int i = 0; i < m; ++i)
      for (int k = std::max(0, i - q); k <= std::min(m - 1, i + q); ++k) {
        const double a = acc[(size_t)i * m + k];
        if (a == 0.0) continue;
        if (k > 0) t[(size_t)i * m + k - 1] += a * y[(size_t)k * m + k - 1];
        if (k + 1 < m) t[(size_t)i * m + k + 1] += a * y[(size_t)k * m + k + 1];
      }
    acc.swap(t);
  }
  Banded G(n);
  for (int i = 0; i < n; ++i)
    for (int o = -3; o <= 3; ++o) {
      const int j = i + o;
      if (j >= 0 && j < n) G.dg[o + 3][i] = coef * acc[(size_t)i * m + j];
    }
  return G;
}
}  // namespace

void plbo_fock_isometry(int D, int d, const double* p, int levels, std::vector<cd>& W) {
  const int n = levels;
  const cd I(0.0, 1.0);
  const cd al(p[0], p[1]);
  const cd z = std::polar(p[2], p[3]);
  // generators (U = exp(GD) exp(GS) R P2 P3 K; applied right to left)
  Banded GD(n), GS(n);
  for (int i = 0; i + 1 < n; ++i) {
    const double s = std::sqrt((double)(i + 1));
    GD.dg[3 + 1][i] = -std::conj(al) * s;  // -alpha^* a: <i|a|i+1>
    GD.dg[3 - 1][i + 1] = al * s;          // alpha a^dag: <i+1|a^dag|i>
  }
  for (int i = 0; i + 2 < n; ++i) {
    const double s = std::sqrt((double)(i + 1) * (i + 2));
    GS.dg[3 + 2][i] = 0.5 * std::conj(z) * s;  // z^* a^2 / 2
    GS.dg[3 - 2][i + 2] = -0.5 * z * s;        // -z a^dag^2 / 2
  }
  const Banded G2 = quad_poly(n, 2, I * (p[5] / 4.0));
  const Banded G3 = quad_poly(n, 3, I * (p[6] / 6.0));
  W.assign((size_t)D * d, 0.0);
  std::vector<cd> x(n);
  for (int m = 0; m < d; ++m) {
    std::fill(x.begin(), x.end(), cd(0.0));
    x[m] = std::exp(I * (p[7] * m * m));  // K
    expmv(G3, x);                          // P3
    expmv(G2, x);                          // P2
    for (int i = 0; i < n; ++i) x[i] *= std::exp(I * (p[4] * i));  // R
    expmv(GS, x);                                                  // S
    expmv(GD, x);                                                  // D
    for (int i = 0; i < D; ++i) W[(size_t)i * d + m] = x[i];
  }
}

// ------------------------------------------------------------------ slot environments (device)
// out[j][n'][n] = sum_{a,b} conj(U_j[a][n'][b]) Y_j[a][n][b] over jobs j; one
// block per (job, n', group of 8 n), FP64 accumulation, fixed-order reduction.
template <typename CT>
__global__ __launch_bounds__(256) void slot_gram_kernel(const SlotJob* __restrict__ jobs, int cl, int d, int cr,
                                                        cf64* __restrict__ out) {
  __shared__ double red[4][16];
  const SlotJob jb = jobs[blockIdx.x];
  const int np = blockIdx.y, n0 = blockIdx.z * 8;
  const int nq = min(8, d - n0);
  const CT* U = (const CT*)jb.U;
  const CT* Y = (const CT*)jb.Y;
  double re[8], im[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) re[q] = im[q] = 0.0;
  const int64_t tot = (int64_t)cl * cr;
  for (int64_t e = threadIdx.x; e < tot; e += 256) {
    const int a = (int)(e / cr), b = (int)(e % cr);
    const CT u = U[((int64_t)a * d + np) * cr + b];
    const double ux = (double)u.x, uy = (double)u.y;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < nq) {
        const CT y = Y[((int64_t)a * d + n0 + q) * cr + b];
        re[q] += ux * (double)y.x + uy * (double)y.y;
        im[q] += ux * (double)y.y - uy * (double)y.x;
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double r = wave_reduce_sum(re[q]), i = wave_reduce_sum(im[q]);
    if (lane == 0) {
      red[wave][2 * q] = r;
      red[wave][2 * q + 1] = i;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nq) {
    const int t = threadIdx.x;
    const double v = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    double* o = (double*)(out + ((int64_t)blockIdx.x * d + np) * d + n0 + (t >> 1));
    o[t & 1] = v;
  }
}

hipError_t launch_slot_gram(int sprec, const SlotJob* d_jobs, int njobs, int cl, int d, int cr, cf64* out,
                            hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  dim3 grid(njobs, d, (d + 7) / 8);
  if (sprec == PREC_FP64)
    hipLaunchKernelGGL(slot_gram_kernel<cf64>, grid, dim3(256), 0, st, d_jobs, cl, d, cr, out);
  else
    hipLaunchKernelGGL(slot_gram_kernel<cf32>, grid, dim3(256), 0, st, d_jobs, cl, d, cr, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ host entry points
extern "C" tn_status tn_plbo_ops(int32_t d, const double* params, double a_ss, double b_ss, double g_ss,
                                 double* ops, double* dops) {
  if (d < 1 || d > 64 || !params || !ops) return TN_EINVAL;
  for (int j = 0; j < NP; ++j)
    if (!std::isfinite(params[j])) return TN_EINVAL;
  if (!std::isfinite(a_ss) || !std::isfinite(b_ss) || !std::isfinite(g_ss)) return TN_EINVAL;
  try {
    std::vector<cd> o, g;
    plbo_local_ops(d, params, a_ss, b_ss, g_ss, o, dops ? &g : nullptr);
    std::memcpy(ops, o.data(), o.size() * sizeof(cd));
    if (dops) std::memcpy(dops, g.data(), g.size() * sizeof(cd));
  } catch (...) {
    return TN_EINVAL;
  }
  return TN_OK;
}

extern "C" tn_status tn_plbo_fock_isometry(int32_t D, int32_t d, const double* params, int32_t levels, double* iso) {
  if (d < 1 || D < d || D > 4096 || !params || !iso) return TN_EINVAL;
  if (levels < D || levels > 8192) return TN_EINVAL;
  for (int j = 0; j < NP; ++j)
    if (!std::isfinite(params[j])) return TN_EINVAL;
  try {
    std::vector<cd> W;
    plbo_fock_isometry(D, d, params, levels, W);
    std::memcpy(iso, W.data(), W.size() * sizeof(cd));
  } catch (...) {
    return TN_EINVAL;
  }
  return TN_OK;
}

extern "C" tn_status tn_plbo_minimize(int32_t d, const double* G, double a_ss, double b_ss, double g_ss,
                                      const tn_plbo_opts* opts, double* params, double* energy) {
  if (d < 1 || d > 64 || !G || !opts || !params || !energy) return TN_EINVAL;
  if (opts->steps < 0 || !(opts->lr > 0.0) || (opts->optimizer != TN_PLBO_ADAM && opts->optimizer != TN_PLBO_LBFGS))
    return TN_EINVAL;
  if (!(opts->beta1 >= 0.0 && opts->beta1 < 1.0) || !(opts->beta2 >= 0.0 && opts->beta2 < 1.0) || !(opts->eps > 0.0))
    return TN_EINVAL;
  for (int j = 0; j < NP; ++j)
    if (!std::isfinite(params[j])) return TN_EINVAL;
  try {
    std::vector<cd> Gh((size_t)(NOPS + 1) * d * d);
    std::memcpy(Gh.data(), G, Gh.size() * sizeof(cd));
    const PlboSite S{d, a_ss, b_ss, g_ss, &Gh};
    double m[NP] = {}, v[NP] = {};
    int t = 0;
    plbo_optimise(S, *opts, params, m, v, &t);
    *energy = plbo_site_energy(S, params, nullptr);
  } catch (...) {
    return TN_EINVAL;
  }
  return TN_OK;
}

// Effective cutoff of the basis (eq. Effectivecutoff): the smallest D at which
// the first d basis vectors, cut to D Fock rows, are orthonormal within tol.
extern "C" tn_status tn_plbo_effective_cutoff(int32_t d, const double* params, int32_t D_max, double tol,
                                              int32_t* D_eff) {
  if (d < 1 || D_max < d || D_max > 4096 || !params || !D_eff || !(tol > 0.0)) return TN_EINVAL;
  for (int j = 0; j < NP; ++j)
    if (!std::isfinite(params[j])) return TN_EINVAL;
  try {
    std::vector<cd> W;
    plbo_fock_isometry(D_max, d, params, D_max + 192, W);
    std::vector<cd> G((size_t)d * d, 0.0);
    *D_eff = -1;
    for (int D = 1; D <= D_max; ++D) {
      const cd* row = W.data() + (size_t)(D - 1) * d;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) G[(size_t)i * d + j] += std::conj(row[i]) * row[j];
      if (D < d) continue;
      double dev = 0.0;
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) dev = std::max(dev, std::abs(G[(size_t)i * d + j] - (i == j ? 1.0 : 0.0)));
      if (dev <= tol) {
        *D_eff = D;
        break;
      }
    }
  } catch (...) {
    return TN_ENOMEM;
  }
  return TN_OK;
}
