// Reference oracle for the sparse wavefunction circuit solver (SWCS) used in
// ADAPT-VQE (arXiv 2411.07920).  TEST INFRASTRUCTURE ONLY: the tests, the
// smoke check and the CPU-baseline leg of the benchmark call it; the product
// path never does.  It shares no code with the HIP library.
//
// Plain, slow and meant to be checked by eye against the paper and textbook
// formulas: ordered std::map states, operator strings applied one ladder
// operator at a time, Slater-Condon rules written out, no blocking or fusion.
//
// Conventions (the paper is silent on them):
//   * spin-orbital P = 2p + sigma, bit P of a uint64 key = occupation;
//   * |D> = a+_{P1} ... a+_{Pk} |0> with P1 < ... < Pk, so a ladder operator on
//     spin-orbital P picks up (-1)^(number of occupied spin-orbitals below P);
//   * pool row (P, Q, R, S): double T = a+_P a+_Q a_S a_R; row (P, Q, -1, -1):
//     single T = a+_P a_Q; generator A = T - T^dagger.
//
// Functions (each names the passage it follows):
//   orc_hmat            Slater-Condon matrix elements (Szabo & Ostlund, cited
//                       in Sec. III) of H = sum h a+a + 1/2 sum (pq|rs) a+a+aa.
//   orc_apply_ansatz    Eq. (1)-(3): product of exp(theta A) applied in list
//                       order, each unitary evaluated exactly (Sec. II.B), the
//                       state pruned after every unitary (Fig. 1): either by
//                       amplitude magnitude |c| < eps (the alternative named at
//                       the end of the first SWCS paragraph) or by keeping the
//                       N_CUT largest magnitudes (the primary rule there).
//   orc_energy          Rayleigh quotient <psi|H|psi>/<psi|psi>.
//   orc_pool_gradients  Step 4 of the ADAPT loop (Sec. II.C): derivative of the
//                       energy with respect to the parameter of each pool
//                       operator appended at the end of the ansatz,
//                       <psi|[H, A_k]|psi>/<psi|psi>.
//   orc_param_gradients Analytic gradients (Sec. II.B) for the VQE step: the
//                       derivative of E with each gate's kept support frozen
//                       (truncation is then a fixed projection), computed by
//                       the adjoint (reverse) recursion over stored states.
//   orc_energy_frozen   Energy of the chain with every gate's support frozen to
//                       that of a reference run (masked finite differences).
//   orc_*_gen_*         The same for chains of spin-complemented generators
//                       (Sec. III): a generator is a pool row, or two rows with
//                       one shared parameter, G = A_k1 + s A_k2.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <unordered_map>
#include <vector>
#include <algorithm>
#include <utility>

typedef std::map<uint64_t, double> State;  // ordered: sums run in key order

struct Problem {
  int n;        // spatial orbitals
  int nso;      // spin-orbitals = 2n
  int n_alpha, n_beta;
  std::vector<double> h;    // n*n
  std::vector<double> eri;  // n^4, (pq|rs) chemists' notation
  double ecore;
};

// ---------------------------------------------------------------- ladder ops
// Number of occupied spin-orbitals strictly below P, counted one by one.
static int occupied_below(uint64_t D, int P) {
  int count = 0;
  for (int Q = 0; Q < P; ++Q)
    if ((D >> Q) & 1ULL) ++count;
  return count;
}

// a_P |D>: returns 0 if P is empty, else the sign; D is updated in place.
static int annihilate(uint64_t& D, int P) {
  if (!((D >> P) & 1ULL)) return 0;
  int sign = (occupied_below(D, P) % 2) ? -1 : 1;
  D &= ~(1ULL << P);
  return sign;
}

// a+_P |D>: returns 0 if P is occupied, else the sign; D is updated in place.
static int create(uint64_t& D, int P) {
  if ((D >> P) & 1ULL) return 0;
  int sign = (occupied_below(D, P) % 2) ? -1 : 1;
  D |= (1ULL << P);
  return sign;
}

// Apply an operator string, written left to right as in the formula, to |D>.
// Each entry is (P, is_creator).  The rightmost operator acts first.
static int apply_string(const std::vector<std::pair<int, bool>>& ops, uint64_t& D) {
  int sign = 1;
  for (int t = (int)ops.size() - 1; t >= 0; --t) {
    int s = ops[t].second ? create(D, ops[t].first) : annihilate(D, ops[t].first);
    if (s == 0) return 0;
    sign *= s;
  }
  return sign;
}

// T of a pool row: a+_P a+_Q a_S a_R (double) or a+_P a_Q (single).
static std::vector<std::pair<int, bool>> excitation_string(const int32_t* row) {
  if (row[2] < 0) return {{row[0], true}, {row[1], false}};
  return {{row[0], true}, {row[1], true}, {row[3], false}, {row[2], false}};
}

// T^dagger of a pool row: a+_R a+_S a_Q a_P (double) or a+_Q a_P (single).
static std::vector<std::pair<int, bool>> deexcitation_string(const int32_t* row) {
  if (row[2] < 0) return {{row[1], true}, {row[0], false}};
  return {{row[2], true}, {row[3], true}, {row[1], false}, {row[0], false}};
}

// ---------------------------------------------------------------- integrals
static inline int spin_of(int P) { return P & 1; }
static inline int spatial_of(int P) { return P >> 1; }

// Spin-orbital one-electron integral h_PQ = h_pq delta(sigma_P, sigma_Q).
static double h_so(const Problem& pb, int P, int Q) {
  if (spin_of(P) != spin_of(Q)) return 0.0;
  return pb.h[spatial_of(P) * pb.n + spatial_of(Q)];
}

// Spin-orbital (PQ|RS) = (pq|rs) delta(sigma_P, sigma_Q) delta(sigma_R, sigma_S).
static double eri_so(const Problem& pb, int P, int Q, int R, int S) {
  if (spin_of(P) != spin_of(Q) || spin_of(R) != spin_of(S)) return 0.0;
  int n = pb.n;
  int p = spatial_of(P), q = spatial_of(Q), r = spatial_of(R), s = spatial_of(S);
  return pb.eri[((size_t)(p * n + q) * n + r) * n + s];
}

static std::vector<int> occupied_list(uint64_t D, int nso) {
  std::vector<int> occ;
  for (int P = 0; P < nso; ++P)
    if ((D >> P) & 1ULL) occ.push_back(P);
  return occ;
}

// ---------------------------------------------------------------- Slater-Condon
static double hmat(const Problem& pb, uint64_t bra, uint64_t ket) {
  uint64_t diff = bra ^ ket;
  int ndiff = 0;
  for (int P = 0; P < pb.nso; ++P)
    if ((diff >> P) & 1ULL) ++ndiff;
  if ((diff >> pb.nso) != 0) return 0.0;
  if (ndiff == 0) {
    std::vector<int> occ = occupied_list(ket, pb.nso);
    double e = pb.ecore;
    for (int P : occ) e += h_so(pb, P, P);
    for (int P : occ)
      for (int Q : occ) e += 0.5 * (eri_so(pb, P, P, Q, Q) - eri_so(pb, P, Q, Q, P));
    return e;
  }
  if (ndiff == 2) {
    int I = -1, A = -1;
    for (int P = 0; P < pb.nso; ++P) {
      if (!((diff >> P) & 1ULL)) continue;
      if ((ket >> P) & 1ULL) I = P; else A = P;
    }
    if (I < 0 || A < 0) return 0.0;  // particle number differs
    uint64_t D = ket;
    int gamma = apply_string({{A, true}, {I, false}}, D);
    if (gamma == 0 || D != bra) return 0.0;
    double v = h_so(pb, A, I);
    for (int Q : occupied_list(ket, pb.nso))
      v += eri_so(pb, A, I, Q, Q) - eri_so(pb, A, Q, Q, I);
    return gamma * v;
  }
  if (ndiff == 4) {
    std::vector<int> holes, parts;
    for (int P = 0; P < pb.nso; ++P) {
      if (!((diff >> P) & 1ULL)) continue;
      if ((ket >> P) & 1ULL) holes.push_back(P); else parts.push_back(P);
    }
    if (holes.size() != 2 || parts.size() != 2) return 0.0;
    int I = holes[0], J = holes[1], A = parts[0], B = parts[1];
    uint64_t D = ket;
    int gamma = apply_string({{A, true}, {B, true}, {J, false}, {I, false}}, D);
    if (gamma == 0 || D != bra) return 0.0;
    double v = eri_so(pb, A, I, B, J) - eri_so(pb, A, J, B, I);
    return gamma * v;
  }
  return 0.0;
}

// All determinants reachable from D by moving zero, one or two electrons
// (any spins; spin-violating ones get a zero matrix element).  Includes D.
static std::vector<uint64_t> neighbourhood(const Problem& pb, uint64_t D) {
  std::vector<int> occ, vir;
  for (int P = 0; P < pb.nso; ++P) {
    if ((D >> P) & 1ULL) occ.push_back(P); else vir.push_back(P);
  }
  std::vector<uint64_t> out;
  out.push_back(D);
  for (int i : occ)
    for (int a : vir) out.push_back(D ^ (1ULL << i) ^ (1ULL << a));
  for (size_t x = 0; x < occ.size(); ++x)
    for (size_t y = x + 1; y < occ.size(); ++y)
      for (size_t u = 0; u < vir.size(); ++u)
        for (size_t w = u + 1; w < vir.size(); ++w)
          out.push_back(D ^ (1ULL << occ[x]) ^ (1ULL << occ[y]) ^ (1ULL << vir[u]) ^
                        (1ULL << vir[w]));
  return out;
}

// sigma_P(D) = sum_{D' in psi} H_{D D'} psi(D') for every D in psi.
static State sigma_projected(const Problem& pb, const State& psi) {
  State sig;
  for (const auto& kv : psi) {
    double acc = 0.0;
    for (uint64_t Dp : neighbourhood(pb, kv.first)) {
      auto it = psi.find(Dp);
      if (it == psi.end()) continue;
      acc += hmat(pb, kv.first, Dp) * it->second;
    }
    sig[kv.first] = acc;
  }
  return sig;
}

// sigma(X) = sum_{D' in psi} H_{X D'} psi(D') for every X connected to psi.
static std::unordered_map<uint64_t, double> sigma_external(const Problem& pb, const State& psi) {
  std::unordered_map<uint64_t, double> sig;
  for (const auto& kv : psi)
    for (uint64_t X : neighbourhood(pb, kv.first)) {
      double hx = hmat(pb, X, kv.first);
      if (hx != 0.0) sig[X] += hx * kv.second;
    }
  return sig;
}

static void energy_of(const Problem& pb, const State& psi, double* numer, double* norm2, double* E) {
  State sig = sigma_projected(pb, psi);
  double nu = 0.0, no = 0.0;
  for (const auto& kv : psi) {
    nu += kv.second * sig[kv.first];
    no += kv.second * kv.second;
  }
  *numer = nu;
  *norm2 = no;
  *E = nu / no;
}

// ---------------------------------------------------------------- gates
// A |psi> for A = T - T^dagger.
static State apply_generator(const int32_t* row, const State& psi) {
  State out;
  auto Tstr = excitation_string(row);
  auto Tdstr = deexcitation_string(row);
  for (const auto& kv : psi) {
    uint64_t D = kv.first;
    int s = apply_string(Tstr, D);
    if (s) out[D] += s * kv.second;
    D = kv.first;
    s = apply_string(Tdstr, D);
    if (s) out[D] -= s * kv.second;
  }
  return out;
}

// exp(theta A) |psi> evaluated exactly.  Because T^2 = 0 and the index sets of
// T are disjoint, A^3 = -A and exp(theta A) = 1 + sin(theta) A +
// (1 - cos(theta)) A^2; on each pair (D, X = T D) with <X|T|D> = s it is the
// rotation psi'(D) = c psi(D) - s sn psi(X), psi'(X) = c psi(X) + s sn psi(D),
// and it leaves every determinant outside such pairs unchanged.  Partners
// absent from psi count as zero.  c = cos(theta), sn = sin(theta).
static State apply_gate(const int32_t* row, double c, double sn, const State& psi) {
  auto Tstr = excitation_string(row);
  auto Tdstr = deexcitation_string(row);
  // Collect every pair (source D, image X, sign s) touching psi.
  std::map<uint64_t, std::pair<uint64_t, int>> pairs;  // D -> (X, s)
  std::set<uint64_t> in_pair;
  for (const auto& kv : psi) {
    uint64_t X = kv.first;
    int s = apply_string(Tstr, X);
    if (s) {
      pairs[kv.first] = {X, s};
      continue;
    }
    uint64_t D = kv.first;
    int sd = apply_string(Tdstr, D);
    if (sd) {
      // kv.first = X is the image of D; <X|T|D> equals <D|T^dagger|X> = sd.
      pairs[D] = {kv.first, sd};
    }
  }
  State out;
  for (const auto& kv : psi) out[kv.first] = kv.second;  // untouched copy
  for (const auto& pr : pairs) {
    uint64_t D = pr.first, X = pr.second.first;
    double s = (double)pr.second.second;
    auto iD = psi.find(D);
    auto iX = psi.find(X);
    double a = (iD == psi.end()) ? 0.0 : iD->second;
    double b = (iX == psi.end()) ? 0.0 : iX->second;
    out[D] = c * a - s * (sn * b);
    out[X] = c * b + s * (sn * a);
  }
  return out;
}

// Drop amplitudes with |c| < eps (strict); eps = 0 keeps everything.
static State truncate_eps(const State& psi, double eps, double* dropped_sq) {
  State out;
  double d2 = 0.0;
  for (const auto& kv : psi) {
    if (std::fabs(kv.second) < eps) d2 += kv.second * kv.second;
    else out.insert(kv);
  }
  if (dropped_sq) *dropped_sq += d2;
  return out;
}

// Keep the ncut largest |c|; ties keep the smaller key.
static State truncate_ncut(const State& psi, int64_t ncut, double* dropped_sq) {
  if ((int64_t)psi.size() <= ncut) return psi;
  std::vector<std::pair<double, uint64_t>> v;
  for (const auto& kv : psi) v.push_back({std::fabs(kv.second), kv.first});
  std::sort(v.begin(), v.end(), [](const std::pair<double, uint64_t>& x,
                                   const std::pair<double, uint64_t>& y) {
    if (x.first != y.first) return x.first > y.first;
    return x.second < y.second;
  });
  State out;
  double d2 = 0.0;
  for (size_t t = 0; t < v.size(); ++t) {
    double amp = psi.at(v[t].second);
    if ((int64_t)t < ncut) out[v[t].second] = amp;
    else d2 += amp * amp;
  }
  if (dropped_sq) *dropped_sq += d2;
  return out;
}

static State truncate(const State& psi, double eps, int64_t ncut, double* dropped_sq) {
  if (ncut > 0) return truncate_ncut(psi, ncut, dropped_sq);
  return truncate_eps(psi, eps, dropped_sq);
}

// psi_i = P(U_{k_i}(theta_i) psi_{i-1}), i = 1..M, starting from the reference.
static std::vector<State> forward_states(const int32_t* pool, const int32_t* ops,
                                         const double* theta, int64_t M, double eps,
                                         int64_t ncut, uint64_t ref, double* dropped_sq) {
  std::vector<State> st;
  State psi;
  psi[ref] = 1.0;
  st.push_back(psi);
  for (int64_t i = 0; i < M; ++i) {
    const int32_t* row = pool + 4 * (int64_t)ops[i];
    double c = std::cos(theta[i]), sn = std::sin(theta[i]);
    psi = truncate(apply_gate(row, c, sn, psi), eps, ncut, dropped_sq);
    st.push_back(psi);
  }
  return st;
}

static double dot(const State& x, const State& y) {
  double acc = 0.0;
  for (const auto& kv : x) {
    auto it = y.find(kv.first);
    if (it != y.end()) acc += kv.second * it->second;
  }
  return acc;
}

// ---------------------------------------------------------------- generators
// Spin-complemented generator G = A1 + s A2 (A_i = T_i - T_i^dagger of pool
// rows 1 and 2, s = +-1) with one parameter theta (Sec. III).
//
// When T1 and T2 act on disjoint spin-orbitals they commute and
// exp(theta G) = exp(theta A1) exp(s theta A2): the generator is applied as
// those two unitaries (row 1 first), each followed by pruning.
//
// When T1 and T2 share their created pair (or their annihilated pair) and
// are otherwise disjoint -- an opposite-spin double with p = q (or r = s) and
// its complement -- G connects each determinant to at most two others, and
// only in one of two shapes:
//   * a pair {D, X}: exactly one of T1, T2 (or their adjoints) acts on D and
//     X has no other connection -- the usual rotation at angle theta (at
//     s theta for row 2);
//   * a star {C, L1, L2}: T1 and T2 both act on C (or both adjoints do), with
//     G C = alpha L1 + beta L2 (alpha, beta = +-1), G L1 = -alpha C,
//     G L2 = -beta C.  G^2 C = -2 C, so on the star exp(theta G) rotates C
//     and u = (alpha x1 + beta x2) / sqrt(2) at frequency sqrt(2) theta and
//     leaves the leaf combination orthogonal to u unchanged:
//       xc' = c2 xc - s2 u,   u' = s2 xc + c2 u,
//       xi' = xi + (coef_i / sqrt(2)) (u' - u),  coef_1 = alpha, coef_2 = beta,
//     with c2 = cos(sqrt(2) theta), s2 = sin(sqrt(2) theta).

// Pool row's operator acting on D: +1 T, -1 T^dagger, 0 neither (it cannot
// be both).  *X receives the image, *ph the sign of <X|T|D> or <X|T^dagger|D>.
static int row_action(const int32_t* row, uint64_t D, uint64_t* X, int* ph) {
  uint64_t Y = D;
  int s = apply_string(excitation_string(row), Y);
  if (s) {
    *X = Y;
    *ph = s;
    return 1;
  }
  Y = D;
  s = apply_string(deexcitation_string(row), Y);
  if (s) {
    *X = Y;
    *ph = s;
    return -1;
  }
  return 0;
}

static bool rows_share_spin_orbitals(const int32_t* r1, const int32_t* r2) {
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      if (r1[a] >= 0 && r1[a] == r2[b]) return true;
  return false;
}

// <X|G|D> restricted to one row: the G-coefficient of X in G|D> for the row
// acting on D (act = +1: +<X|T|D>, act = -1: -<X|T^dagger|D>), times its factor.
static double gen_coef(int act, int ph, double factor) { return factor * (act > 0 ? ph : -ph); }

// exp(theta G) for two rows sharing their created (or annihilated) pair.
static State apply_star_gate(const int32_t* r1, const int32_t* r2, double sg, double c, double sn,
                             double c2, double s2, double rt, const State& psi) {
  State out = psi;
  std::set<uint64_t> done;  // components already rotated, by their first member
  auto val = [&](uint64_t k) {
    auto it = psi.find(k);
    return it == psi.end() ? 0.0 : it->second;
  };
  for (const auto& kv : psi) {
    const uint64_t D = kv.first;
    uint64_t X1 = 0, X2 = 0;
    int p1 = 0, p2 = 0;
    const int a1 = row_action(r1, D, &X1, &p1);
    const int a2 = row_action(r2, D, &X2, &p2);
    if (!a1 && !a2) continue;
    // the component: a star centred at C, or a pair
    uint64_t C = 0, L1 = 0, L2 = 0;
    double al = 0.0, be = 0.0;
    bool star = false;
    if (a1 && a2) {
      star = true;
      C = D, L1 = X1, L2 = X2;
      al = gen_coef(a1, p1, 1.0);
      be = gen_coef(a2, p2, sg);
    } else {
      const int32_t* row = a1 ? r1 : r2;
      const int32_t* other = a1 ? r2 : r1;
      const uint64_t P = a1 ? X1 : X2;
      uint64_t Q = 0;
      int pq = 0, po = 0;
      uint64_t Po = 0;
      // the partner is a star centre if the other row acts on it as well
      if (row_action(other, P, &Po, &po)) {
        star = true;
        C = P;
        int pr = 0;
        const int ar = row_action(row, C, &Q, &pr);
        const int ao = row_action(other, C, &Po, &po);
        L1 = a1 ? Q : Po;
        L2 = a1 ? Po : Q;
        al = a1 ? gen_coef(ar, pr, 1.0) : gen_coef(ao, po, 1.0);
        be = a1 ? gen_coef(ao, po, sg) : gen_coef(ar, pr, sg);
      } else {
        // pair: the source is the member T acts on
        const int act = a1 ? a1 : a2;
        const int ph = a1 ? p1 : p2;
        const uint64_t src = act > 0 ? D : P;
        const uint64_t dst = act > 0 ? P : D;
        if (done.count(src)) continue;
        done.insert(src);
        const double f = a1 ? 1.0 : sg;  // row 2 turns by s theta
        const double sn_r = f * sn;
        const double a = val(src), b = val(dst);
        const double sp = (double)ph;  // <dst|T|src> either way
        out[src] = c * a - sp * (sn_r * b);
        out[dst] = c * b + sp * (sn_r * a);
        continue;
      }
      (void)pq;
    }
    if (!star || done.count(C)) continue;
    done.insert(C);
    const double xc = val(C), x1 = val(L1), x2 = val(L2);
    const double u = (al * x1 + be * x2) * rt;
    const double nc = c2 * xc - s2 * u;
    const double nu = s2 * xc + c2 * u;
    const double du = nu - u;
    out[C] = nc;
    out[L1] = x1 + al * (rt * du);
    out[L2] = x2 + be * (rt * du);
  }
  return out;
}

// One generator of a chain: pool rows r1 and r2 (r2 == NULL: the single row
// r1), factor sg.
struct Gen {
  const int32_t* r1;
  const int32_t* r2;
  double sg;
};

static bool gen_is_star(const Gen& g) { return g.r2 && rows_share_spin_orbitals(g.r1, g.r2); }

// exp(theta G) psi followed by pruning (after each unitary of a commuting pair).
static State apply_gen(const Gen& g, double theta, double eps, int64_t ncut, const State& psi,
                       double* dropped_sq) {
  const double c = std::cos(theta), sn = std::sin(theta);
  if (!g.r2) return truncate(apply_gate(g.r1, c, sn, psi), eps, ncut, dropped_sq);
  if (!gen_is_star(g)) {
    State mid = truncate(apply_gate(g.r1, c, sn, psi), eps, ncut, dropped_sq);
    return truncate(apply_gate(g.r2, c, g.sg * sn, mid), eps, ncut, dropped_sq);
  }
  const double w = std::sqrt(2.0) * theta;
  return truncate(apply_star_gate(g.r1, g.r2, g.sg, c, sn, std::cos(w), std::sin(w), 1.0 / std::sqrt(2.0), psi),
                  eps, ncut, dropped_sq);
}

// G psi = A1 psi + s A2 psi.
static State apply_gen_sum(const Gen& g, const State& psi) {
  State out = apply_generator(g.r1, psi);
  if (g.r2)
    for (const auto& kv : apply_generator(g.r2, psi)) out[kv.first] += g.sg * kv.second;
  return out;
}

static std::vector<Gen> gen_list(const int32_t* pool, const int32_t* gens, int64_t M) {
  std::vector<Gen> v;
  for (int64_t i = 0; i < M; ++i) {
    Gen g;
    g.r1 = pool + 4 * (int64_t)gens[3 * i];
    g.r2 = gens[3 * i + 1] >= 0 ? pool + 4 * (int64_t)gens[3 * i + 1] : nullptr;
    g.sg = (double)gens[3 * i + 2];
    v.push_back(g);
  }
  return v;
}

// ---------------------------------------------------------------- C ABI
struct OracleState {
  State psi;
};

extern "C" {

void* orc_problem_create(int n, int n_alpha, int n_beta, const double* h, const double* eri,
                         double ecore) {
  Problem* pb = new Problem;
  pb->n = n;
  pb->nso = 2 * n;
  pb->n_alpha = n_alpha;
  pb->n_beta = n_beta;
  pb->h.assign(h, h + (size_t)n * n);
  pb->eri.assign(eri, eri + (size_t)n * n * n * n);
  pb->ecore = ecore;
  return pb;
}

void orc_problem_destroy(void* p) { delete (Problem*)p; }

void* orc_state_create(const uint64_t* keys, const double* amps, int64_t count) {
  OracleState* s = new OracleState;
  for (int64_t t = 0; t < count; ++t) s->psi[keys[t]] = amps[t];
  return s;
}

void orc_state_destroy(void* s) { delete (OracleState*)s; }

int64_t orc_state_size(void* s) { return (int64_t)((OracleState*)s)->psi.size(); }

// Sorted by key, ascending.
void orc_state_export(void* s, uint64_t* keys, double* amps) {
  int64_t t = 0;
  for (const auto& kv : ((OracleState*)s)->psi) {
    keys[t] = kv.first;
    amps[t] = kv.second;
    ++t;
  }
}

double orc_hmat(void* p, uint64_t bra, uint64_t ket) { return hmat(*(Problem*)p, bra, ket); }

// One gate on a state (no truncation); c and sn as given.
void* orc_apply_gate(void* s, const int32_t* row, double c, double sn) {
  OracleState* out = new OracleState;
  out->psi = apply_gate(row, c, sn, ((OracleState*)s)->psi);
  return out;
}

// One gate followed by truncation, on a state.
void* orc_apply_gate_truncate(void* s, const int32_t* row, double c, double sn, double eps,
                              int64_t ncut, double* dropped_sq) {
  OracleState* out = new OracleState;
  *dropped_sq = 0.0;
  out->psi = truncate(apply_gate(row, c, sn, ((OracleState*)s)->psi), eps, ncut, dropped_sq);
  return out;
}

// A|psi> for the generator of a pool row.
void* orc_apply_generator(void* s, const int32_t* row) {
  OracleState* out = new OracleState;
  out->psi = apply_generator(row, ((OracleState*)s)->psi);
  return out;
}

// Full ansatz from the reference.  ncut > 0 selects N_CUT pruning, else eps.
void* orc_apply_ansatz(const int32_t* pool, const int32_t* ops, const double* theta, int64_t M,
                       double eps, int64_t ncut, uint64_t ref, double* dropped_sq) {
  double d2 = 0.0;
  std::vector<State> st = forward_states(pool, ops, theta, M, eps, ncut, ref, &d2);
  if (dropped_sq) *dropped_sq = d2;
  OracleState* out = new OracleState;
  out->psi = st.back();
  return out;
}

void orc_energy(void* p, void* s, double* numer, double* norm2, double* E) {
  energy_of(*(Problem*)p, ((OracleState*)s)->psi, numer, norm2, E);
}

// sigma_P on the support of psi, exported sorted by key.
void orc_sigma_projected(void* p, void* s, double* out) {
  State sig = sigma_projected(*(Problem*)p, ((OracleState*)s)->psi);
  int64_t t = 0;
  for (const auto& kv : sig) out[t++] = kv.second;
}

// sigma(X) for given keys X (any determinants): sum_{D' in psi} H_{X D'} psi(D').
void orc_sigma_at(void* p, void* s, const uint64_t* X, int64_t count, double* out) {
  const Problem& pb = *(Problem*)p;
  const State& psi = ((OracleState*)s)->psi;
  for (int64_t t = 0; t < count; ++t) {
    double acc = 0.0;
    for (uint64_t Dp : neighbourhood(pb, X[t])) {
      auto it = psi.find(Dp);
      if (it != psi.end()) acc += hmat(pb, X[t], Dp) * it->second;
    }
    out[t] = acc;
  }
}

// g_k = <psi|[H, A_k]|psi> / <psi|psi> = 2 <H psi | A_k psi> / <psi|psi> for
// real psi, symmetric H and antisymmetric A_k.  subset == NULL means all K.
void orc_pool_gradients(void* p, void* s, const int32_t* pool, int64_t K, const int32_t* subset,
                        int64_t n_subset, double* g) {
  const Problem& pb = *(Problem*)p;
  const State& psi = ((OracleState*)s)->psi;
  std::unordered_map<uint64_t, double> sig = sigma_external(pb, psi);
  double norm2 = 0.0;
  for (const auto& kv : psi) norm2 += kv.second * kv.second;
  int64_t count = subset ? n_subset : K;
  for (int64_t t = 0; t < count; ++t) {
    int64_t k = subset ? subset[t] : t;
    State Apsi = apply_generator(pool + 4 * k, psi);
    double acc = 0.0;
    for (const auto& kv : Apsi) {
      auto it = sig.find(kv.first);
      if (it != sig.end()) acc += it->second * kv.second;
    }
    g[t] = 2.0 * acc / norm2;
  }
}

// Frozen-support adjoint.  E = N/S with N = <psi|H|psi>, S = <psi|psi>;
// dE/dpsi_M = (2/S)(H psi_M - E psi_M) on the kept support S_M; each gate
// psi_i = P_i U_i psi_{i-1} passes back mu_{i-1} = P_{S_{i-1}} U_i^T mu_i and
// contributes dE/dtheta_i = <mu_i | P_i A U_i psi_{i-1}> = <U_i(-theta_i) mu_i |
// A psi_{i-1}> (A commutes with U_i and mu_i lies in S_i).
void orc_param_gradients(void* p, const int32_t* pool, const int32_t* ops, const double* theta,
                         int64_t M, double eps, int64_t ncut, uint64_t ref, double* dE,
                         double* E_out) {
  const Problem& pb = *(Problem*)p;
  std::vector<State> st = forward_states(pool, ops, theta, M, eps, ncut, ref, nullptr);
  const State& psiM = st.back();
  double numer, norm2, E;
  energy_of(pb, psiM, &numer, &norm2, &E);
  State sig = sigma_projected(pb, psiM);
  State mu;
  for (const auto& kv : psiM) mu[kv.first] = (2.0 / norm2) * (sig[kv.first] - E * kv.second);
  for (int64_t i = M - 1; i >= 0; --i) {
    const int32_t* row = pool + 4 * (int64_t)ops[i];
    double c = std::cos(theta[i]), sn = std::sin(theta[i]);
    State nu = apply_gate(row, c, -sn, mu);  // U(-theta) = U(theta)^T
    State Apsi = apply_generator(row, st[i]);
    dE[i] = dot(nu, Apsi);
    State next;
    for (const auto& kv : st[i]) {
      auto it = nu.find(kv.first);
      next[kv.first] = (it == nu.end()) ? 0.0 : it->second;
    }
    mu = next;
  }
  if (E_out) *E_out = E;
}

// Energy of the chain at parameters theta_eval with every gate's support frozen
// to the support produced by the run at theta_ref (truncation replaced by the
// fixed projection onto that support).
double orc_energy_frozen(void* p, const int32_t* pool, const int32_t* ops,
                         const double* theta_ref, const double* theta_eval, int64_t M, double eps,
                         int64_t ncut, uint64_t ref) {
  const Problem& pb = *(Problem*)p;
  std::vector<State> st = forward_states(pool, ops, theta_ref, M, eps, ncut, ref, nullptr);
  State psi;
  psi[ref] = 1.0;
  for (int64_t i = 0; i < M; ++i) {
    const int32_t* row = pool + 4 * (int64_t)ops[i];
    State u = apply_gate(row, std::cos(theta_eval[i]), std::sin(theta_eval[i]), psi);
    State kept;
    for (const auto& kv : st[i + 1]) {
      auto it = u.find(kv.first);
      kept[kv.first] = (it == u.end()) ? 0.0 : it->second;
    }
    psi = kept;
  }
  double numer, norm2, E;
  energy_of(pb, psi, &numer, &norm2, &E);
  return E;
}

// One generator on a state: gens3 = (k1, k2, s) rows of `pool` (k2 < 0: row
// k1 alone), then pruning.
void* orc_apply_gen(void* st, const int32_t* pool, const int32_t* gens3, double theta, double eps,
                    int64_t ncut, double* dropped_sq) {
  std::vector<Gen> g = gen_list(pool, gens3, 1);
  OracleState* out = new OracleState;
  double d2 = 0.0;
  out->psi = apply_gen(g[0], theta, eps, ncut, ((OracleState*)st)->psi, &d2);
  if (dropped_sq) *dropped_sq = d2;
  return out;
}

// G|psi> of one generator.
void* orc_apply_gen_sum(void* st, const int32_t* pool, const int32_t* gens3) {
  std::vector<Gen> g = gen_list(pool, gens3, 1);
  OracleState* out = new OracleState;
  out->psi = apply_gen_sum(g[0], ((OracleState*)st)->psi);
  return out;
}

// Chain of M generators gens[M x 3] from the reference, generator 0 first.
void* orc_apply_gen_ansatz(const int32_t* pool, const int32_t* gens, const double* theta, int64_t M,
                           double eps, int64_t ncut, uint64_t ref) {
  std::vector<Gen> g = gen_list(pool, gens, M);
  State psi;
  psi[ref] = 1.0;
  for (int64_t i = 0; i < M; ++i) psi = apply_gen(g[(size_t)i], theta[i], eps, ncut, psi, nullptr);
  OracleState* out = new OracleState;
  out->psi = psi;
  return out;
}

// Frozen-support adjoint over a chain of generators.  A generator applied as
// two commuting unitaries is two steps of the recursion (the second at angle
// s theta, whose derivative enters with the factor s); an overlapping pair is
// one step, nu = exp(-theta G) mu, dE/dtheta = <nu | G psi_{i-1}>.
void orc_gen_param_gradients(void* p, const int32_t* pool, const int32_t* gens, const double* theta,
                             int64_t M, double eps, int64_t ncut, uint64_t ref, double* dE,
                             double* E_out) {
  const Problem& pb = *(Problem*)p;
  std::vector<Gen> g = gen_list(pool, gens, M);
  // unit steps: (row or star generator, angle, generator index, factor)
  struct Unit {
    Gen gen;
    double angle;
    int64_t owner;
    double factor;
  };
  std::vector<Unit> units;
  for (int64_t i = 0; i < M; ++i) {
    const Gen& gi = g[(size_t)i];
    if (gi.r2 && !gen_is_star(gi)) {
      units.push_back({Gen{gi.r1, nullptr, 1.0}, theta[i], i, 1.0});
      units.push_back({Gen{gi.r2, nullptr, 1.0}, gi.sg * theta[i], i, gi.sg});
    } else {
      units.push_back({gi, theta[i], i, 1.0});
    }
  }
  std::vector<State> st;
  State psi;
  psi[ref] = 1.0;
  st.push_back(psi);
  for (const Unit& u : units) {
    psi = apply_gen(u.gen, u.angle, eps, ncut, psi, nullptr);
    st.push_back(psi);
  }
  const State& psiN = st.back();
  double numer, norm2, E;
  energy_of(pb, psiN, &numer, &norm2, &E);
  State sig = sigma_projected(pb, psiN);
  State mu;
  for (const auto& kv : psiN) mu[kv.first] = (2.0 / norm2) * (sig[kv.first] - E * kv.second);
  for (int64_t i = 0; i < M; ++i) dE[i] = 0.0;
  for (int64_t j = (int64_t)units.size() - 1; j >= 0; --j) {
    const Unit& u = units[(size_t)j];
    // nu = exp(-angle G) mu without pruning
    State nu = apply_gen(u.gen, -u.angle, 0.0, 0, mu, nullptr);
    dE[u.owner] += u.factor * dot(nu, apply_gen_sum(u.gen, st[(size_t)j]));
    State next;
    for (const auto& kv : st[(size_t)j]) {
      auto it = nu.find(kv.first);
      next[kv.first] = (it == nu.end()) ? 0.0 : it->second;
    }
    mu = next;
  }
  if (E_out) *E_out = E;
}

// Sizes of every intermediate state (|psi_0| .. |psi_M|) of a forward run.
void orc_forward_sizes(const int32_t* pool, const int32_t* ops, const double* theta, int64_t M,
                       double eps, int64_t ncut, uint64_t ref, int64_t* sizes) {
  std::vector<State> st = forward_states(pool, ops, theta, M, eps, ncut, ref, nullptr);
  for (int64_t i = 0; i <= M; ++i) sizes[i] = (int64_t)st[i].size();
}

// <n_P> = sum_D psi(D)^2 [P in D] / <psi|psi>, P = 0..2n-1.
void orc_occupations(void* p, void* s, double* occ) {
  const Problem& pb = *(Problem*)p;
  const State& psi = ((OracleState*)s)->psi;
  double norm2 = 0.0;
  for (int P = 0; P < pb.nso; ++P) occ[P] = 0.0;
  for (const auto& kv : psi) {
    norm2 += kv.second * kv.second;
    for (int P = 0; P < pb.nso; ++P)
      if ((kv.first >> P) & 1ULL) occ[P] += kv.second * kv.second;
  }
  for (int P = 0; P < pb.nso; ++P) occ[P] /= norm2;
}

}  // extern "C"
