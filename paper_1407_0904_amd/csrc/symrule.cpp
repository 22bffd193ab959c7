// Fully symmetric quadrature rules on the reference triangle and tetrahedron.
//
// The paper's kernels carry the small symmetric rules of the form compiler
// (a 3-point rule in the Helmholtz kernel of Listing 1, a 5-point rule in the
// Burgers kernel of Listing 2) but do not print their points. Here such rules
// are found from their definition: a rule is a set of orbits of the symmetry
// group of the simplex (in barycentric coordinates: the centroid; (a,a,1-2a)
// and its permutations; (a,b,1-a-b) and its permutations on triangles; the
// centroid, (a,a,a,1-3a), (a,a,1/2-a,1/2-a) and (a,a,b,1-2a-b) with their
// permutations on tetrahedra), one weight per orbit, and it must integrate
// every monomial x^e, |e| <= degree, exactly. Those moment equations are
// solved by damped Gauss-Newton in long double from a fixed sequence of
// starting points; among the solutions with interior points (and positive
// weights, where the structure has them) the one whose sorted orbit
// parameters are lexicographically smallest is kept, so the rule is
// well-defined. Structures (points, exact degree):
//   triangle  q=1: centroid (1, 1)       q=2: S21 (3, 2)
//             q=3,4: 2 S21 (6, 4)         q=5: centroid + 2 S21 (7, 5)
//             q=6: 2 S21 + S111 (12, 6)
//   tetra     q=1: centroid (1, 1)       q=2: S31 (4, 2)
//             q=3: centroid + S31 (5, 3; the centroid weight is negative)
//             q=4,5: 2 S31 + S22 (14, 5)  q=6: 3 S31 + S211 (24, 6)
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "tables.h"

namespace coffee {

namespace {

using ld = long double;

enum Orbit { S3, S21, S111, S4, S31, S22, S211 };

int orbit_params(Orbit o) { return (o == S3 || o == S4) ? 0 : (o == S111 || o == S211) ? 2 : 1; }

struct Structure {
    int dim, exact;
    std::vector<Orbit> orbits;
    bool positive;  // weights must be positive
};

bool structure_of(int dim, int q, Structure& s) {
    if (dim == 2) {
        switch (q) {
            case 0: case 1: s = {2, 1, {S3}, true}; return true;
            case 2: s = {2, 2, {S21}, true}; return true;
            case 3: case 4: s = {2, 4, {S21, S21}, true}; return true;
            case 5: s = {2, 5, {S3, S21, S21}, true}; return true;
            case 6: s = {2, 6, {S21, S21, S111}, true}; return true;
            default: return false;
        }
    }
    switch (q) {
        case 0: case 1: s = {3, 1, {S4}, true}; return true;
        case 2: s = {3, 2, {S31}, true}; return true;
        case 3: s = {3, 3, {S4, S31}, false}; return true;
        case 4: case 5: s = {3, 5, {S31, S31, S22}, true}; return true;
        case 6: s = {3, 6, {S31, S31, S31, S211}, true}; return true;
        default: return false;
    }
}

// Barycentric points of one orbit (d+1 coordinates each), in a fixed order.
template <typename T>
void orbit_points(Orbit o, const T* p, std::vector<std::vector<T>>& pts) {
    auto perms = [&](std::vector<T> v) {
        std::sort(v.begin(), v.end());
        std::vector<std::vector<T>> out;
        // distinct permutations by position of value classes: enumerate
        // permutations of index order and keep distinct tuples
        std::vector<int> idx(v.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
        do {
            std::vector<T> t(v.size());
            for (size_t i = 0; i < idx.size(); ++i) t[i] = v[idx[i]];
            bool dup = false;
            for (auto& u : out)
                if (u == t) { dup = true; break; }
            if (!dup) out.push_back(t);
        } while (std::next_permutation(idx.begin(), idx.end()));
        for (auto& u : out) pts.push_back(u);
    };
    switch (o) {
        case S3: pts.push_back({T(1) / 3, T(1) / 3, T(1) / 3}); break;
        case S4: pts.push_back({T(0.25), T(0.25), T(0.25), T(0.25)}); break;
        case S21: perms({p[0], p[0], 1 - 2 * p[0]}); break;
        case S111: perms({p[0], p[1], 1 - p[0] - p[1]}); break;
        case S31: perms({p[0], p[0], p[0], 1 - 3 * p[0]}); break;
        case S22: perms({p[0], p[0], T(0.5) - p[0], T(0.5) - p[0]}); break;
        case S211: perms({p[0], p[0], p[1], 1 - 2 * p[0] - p[1]}); break;
    }
}

ld factorial(int n) {
    ld f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

template <typename T>
struct Problem {
    Structure s;
    std::vector<std::vector<int>> mono;  // exponents, |e| <= exact
    std::vector<T> moment;               // exact integrals
    int nunk = 0;

    void init(const Structure& st) {
        s = st;
        nunk = 0;
        for (Orbit o : s.orbits) nunk += orbit_params(o) + 1;
        mono.clear();
        moment.clear();
        const int d = s.dim;
        for (int a = 0; a <= s.exact; ++a)
            for (int b = 0; a + b <= s.exact; ++b)
                for (int c = 0; a + b + c <= s.exact; ++c) {
                    if (d == 2 && c > 0) break;
                    mono.push_back({a, b, c});
                    // integral of x^a y^b (z^c) over the unit simplex
                    const ld m = d == 2 ? factorial(a) * factorial(b) / factorial(a + b + 2)
                                        : factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3);
                    moment.push_back((T)m);
                }
    }

    // Points (Cartesian: barycentric coordinates 1..d) and weights of u.
    void rule(const std::vector<T>& u, std::vector<T>& X, std::vector<T>& W) const {
        X.clear();
        W.clear();
        size_t k = 0;
        for (Orbit o : s.orbits) {
            const int np = orbit_params(o);
            std::vector<std::vector<T>> pts;
            orbit_points<T>(o, &u[k], pts);
            const T w = u[k + np];
            for (auto& b : pts) {
                for (int j = 1; j <= s.dim; ++j) X.push_back(b[j]);
                W.push_back(w);
            }
            k += np + 1;
        }
    }

    void residual(const std::vector<T>& u, std::vector<T>& r) const {
        std::vector<T> X, W;
        rule(u, X, W);
        r.assign(mono.size(), T(0));
        const int d = s.dim, E = s.exact + 1;
        // powers X[p][j]^e, e <= exact
        std::vector<T> pw(W.size() * d * E);
        for (size_t p = 0; p < W.size(); ++p)
            for (int j = 0; j < d; ++j) {
                T* t = &pw[(p * d + j) * E];
                t[0] = 1;
                for (int e = 1; e < E; ++e) t[e] = t[e - 1] * X[p * d + j];
            }
        for (size_t m = 0; m < mono.size(); ++m) {
            T acc = 0;
            for (size_t p = 0; p < W.size(); ++p) {
                T t = W[p];
                for (int j = 0; j < d; ++j) t *= pw[(p * d + j) * E + mono[m][j]];
                acc += t;
            }
            r[m] = (acc - moment[m]) / moment[m];
        }
    }
};

// Damped Gauss-Newton on the scaled moment residuals; returns max |r|.
template <typename T>
T solve(const Problem<T>& P, std::vector<T>& u, T tol2) {
    const int n = P.nunk;
    std::vector<T> r, rp, rm;
    T mu = T(1e-6);
    P.residual(u, r);
    auto norm2 = [](const std::vector<T>& v) {
        T s = 0;
        for (T x : v) s += x * x;
        return s;
    };
    T f = norm2(r);
    for (int it = 0; it < 100 && f > tol2; ++it) {
        const size_t m = r.size();
        std::vector<T> J(m * n);
        for (int j = 0; j < n; ++j) {
            const T h = (sizeof(T) > 8 ? T(1e-9) : T(1e-7)) * std::max(T(1), std::fabs(u[j]));
            std::vector<T> up = u, um = u;
            up[j] += h;
            um[j] -= h;
            P.residual(up, rp);
            P.residual(um, rm);
            for (size_t i = 0; i < m; ++i) J[i * n + j] = (rp[i] - rm[i]) / (2 * h);
        }
        bool improved = false;
        for (int tries = 0; tries < 12 && !improved; ++tries) {
            // (J^T J + mu diag) du = -J^T r
            std::vector<T> A(n * n, 0.0L), g(n, 0.0L);
            for (int a = 0; a < n; ++a) {
                for (int b = 0; b < n; ++b) {
                    T s = 0;
                    for (size_t i = 0; i < m; ++i) s += J[i * n + a] * J[i * n + b];
                    A[a * n + b] = s;
                }
                T s = 0;
                for (size_t i = 0; i < m; ++i) s += J[i * n + a] * r[i];
                g[a] = -s;
            }
            for (int a = 0; a < n; ++a) A[a * n + a] *= (1 + mu);
            // Gaussian elimination with partial pivoting
            std::vector<int> piv(n);
            bool ok = true;
            for (int c = 0; c < n && ok; ++c) {
                int bi = c;
                for (int i = c + 1; i < n; ++i)
                    if (std::fabs(A[i * n + c]) > std::fabs(A[bi * n + c])) bi = i;
                if (!(std::fabs(A[bi * n + c]) > T(1e-290))) { ok = false; break; }
                if (bi != c) {
                    for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[bi * n + k]);
                    std::swap(g[c], g[bi]);
                }
                for (int i = c + 1; i < n; ++i) {
                    const T f2 = A[i * n + c] / A[c * n + c];
                    for (int k = c; k < n; ++k) A[i * n + k] -= f2 * A[c * n + k];
                    g[i] -= f2 * g[c];
                }
            }
            if (!ok) { mu *= 10; continue; }
            std::vector<T> du(n);
            for (int c = n - 1; c >= 0; --c) {
                T s = g[c];
                for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * du[k];
                du[c] = s / A[c * n + c];
            }
            std::vector<T> un = u;
            for (int j = 0; j < n; ++j) un[j] += du[j];
            std::vector<T> rn;
            P.residual(un, rn);
            const T fn = norm2(rn);
            if (std::isfinite((double)fn) && fn < f) {
                u = un;
                r = rn;
                f = fn;
                mu = std::max(mu * T(0.1), T(1e-18));
                improved = true;
            } else {
                mu *= 10;
            }
        }
        if (!improved) break;
    }
    T mx = 0;
    for (T x : r) mx = std::max(mx, std::fabs(x));
    return mx;
}

// Orbit parameters in canonical form (each orbit's parameters reduced to one
// representative, orbits of one type sorted), for comparing solutions.
std::vector<ld> canonical(const Structure& s, std::vector<ld> u) {
    size_t k = 0;
    std::vector<std::pair<int, std::vector<ld>>> orb;
    for (Orbit o : s.orbits) {
        const int np = orbit_params(o);
        std::vector<ld> v(u.begin() + k, u.begin() + k + np + 1);
        if (o == S22) v[0] = std::min(v[0], 0.5L - v[0]);
        if (o == S111) {
            ld t[3] = {v[0], v[1], 1 - v[0] - v[1]};
            std::sort(t, t + 3);
            v[0] = t[0];
            v[1] = t[1];
        }
        if (o == S211) v[1] = std::min(v[1], 1 - 2 * v[0] - v[1]);
        orb.push_back({(int)o, v});
        k += np + 1;
    }
    std::stable_sort(orb.begin(), orb.end(), [](const auto& a, const auto& b) {
        if (a.first != b.first) return a.first < b.first;
        return a.second < b.second;
    });
    std::vector<ld> out;
    for (auto& x : orb) out.insert(out.end(), x.second.begin(), x.second.end());
    return out;
}

bool admissible(const Problem<ld>& P, const std::vector<ld>& u) {
    std::vector<ld> X, W;
    P.rule(u, X, W);
    const int d = P.s.dim;
    for (size_t p = 0; p < W.size(); ++p) {
        ld s = 0;
        for (int j = 0; j < d; ++j) {
            if (!(X[p * d + j] > 1e-12L)) return false;
            s += X[p * d + j];
        }
        if (!(1 - s > 1e-12L)) return false;
        if (P.s.positive && !(W[p] > 0)) return false;
    }
    return true;
}

struct Found {
    std::vector<ld> X, W;
};

bool find_rule(int dim, int q, Found& out) {
    Structure s;
    if (!structure_of(dim, q, s)) return false;
    Problem<double> Pd;
    Pd.init(s);
    Problem<ld> P;
    P.init(s);
    int npts = 0;
    {
        std::vector<ld> X, W, u(P.nunk, 0.1L);
        P.rule(u, X, W);
        npts = (int)W.size();
    }
    const double vol = dim == 2 ? 0.5 : 1.0 / 6;
    // fixed pseudo-random starting points (64-bit LCG); the search runs in
    // double, every converged start is polished in long double
    unsigned long long state = 0x9E3779B97F4A7C15ull ^ (unsigned long long)(dim * 131 + q);
    auto rnd = [&]() {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        return (double)((state >> 11) & ((1ull << 52) - 1)) / (double)(1ull << 52);
    };
    bool have = false;
    std::vector<ld> bestc;
    for (int start = 0; start < 200; ++start) {
        std::vector<double> ud;
        for (Orbit o : s.orbits) {
            switch (o) {
                case S21: ud.push_back(0.5 * rnd()); break;
                case S111: { double a = rnd(), b = rnd() * (1 - a); ud.push_back(a * 0.5); ud.push_back(b * 0.5); break; }
                case S31: ud.push_back(rnd() / 3); break;
                case S22: ud.push_back(0.25 * rnd()); break;
                case S211: { double a = 0.5 * rnd(); ud.push_back(a); ud.push_back((1 - 2 * a) * rnd()); break; }
                default: break;
            }
            ud.push_back(vol / npts * (0.5 + rnd()));
        }
        if (!(solve<double>(Pd, ud, 1e-26) < 1e-11)) continue;
        std::vector<ld> u(ud.begin(), ud.end());
        if (!admissible(P, u)) continue;
        // polish only a candidate that may beat the best rule so far (most
        // starts converge to a rule already found)
        std::vector<ld> c = canonical(s, u);
        if (have) {
            size_t i = 0;
            while (i < c.size() && std::fabs(c[i] - bestc[i]) < 1e-9L) ++i;
            if (i == c.size() || c[i] > bestc[i]) continue;
        }
        if (!(solve<ld>(P, u, 1e-36L) < 1e-15L) || !admissible(P, u)) continue;
        c = canonical(s, u);
        if (!have || c < bestc) {
            bestc = c;
            have = true;
        }
    }
    if (!have) return false;
    // rebuild the rule from the canonical parameters, orbit types in order
    std::vector<Orbit> sorted = s.orbits;
    std::stable_sort(sorted.begin(), sorted.end());
    Structure sc = s;
    sc.orbits = sorted;
    Problem<ld> Pc;
    Pc.init(sc);
    std::vector<ld> u = bestc;
    solve<ld>(Pc, u, 1e-36L);  // polish
    Pc.rule(u, out.X, out.W);
    return true;
}

std::mutex g_mu;
std::map<int, Found> g_rules;  // key dim * 16 + q

const Found* cached_rule(int dim, int q) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int key = dim * 16 + q;
    auto it = g_rules.find(key);
    if (it != g_rules.end()) return &it->second;
    Found f;
    if (!find_rule(dim, q, f)) return nullptr;
    return &(g_rules[key] = f);
}

}  // namespace

int symmetric_rule_size(int dim, int q) {
    Structure s;
    if (!structure_of(dim, q, s)) return -1;
    static const int pts[7] = {1, 3, 6, 1, 4, 6, 12};  // points per orbit type
    int n = 0;
    for (Orbit o : s.orbits) n += pts[o];
    return n;
}

bool symmetric_rule(int dim, int q, long double* X, long double* W) {
    const Found* f = cached_rule(dim, q);
    if (!f) return false;
    std::copy(f->X.begin(), f->X.end(), X);
    std::copy(f->W.begin(), f->W.end(), W);
    return true;
}

}  // namespace coffee
