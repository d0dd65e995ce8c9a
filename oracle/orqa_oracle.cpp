// ORQA reference oracle: plain, single-threaded, FP64, std::map.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark use it.  It shares no code with the HIP library.
//
// What it computes (paper, Methods and Appendix A):
//  * A Pauli string is a multi-index I = I_1|...|I_n of 2-bit codes,
//    00 = id, 01 = sigma_x, 10 = sigma_y, 11 = sigma_z (Methods, Eq. (1)).
//    Code value 1,2,3 is therefore directly the Levi-Civita index x,y,z.
//  * sigma_I sigma_J = i^{B(I,J)} sigma_{I xor J}, with
//    B(I,J) = sum_i b(I_i,J_i), b = 0 if either code is 00, otherwise
//    b(I_i,J_i) = sum_k eps_{I_i J_i k} (Eq. orqaproduct).
//  * A gate (J, theta) is exp(-i theta sigma_J / 2); conjugating O by it
//    changes the coefficient of sigma_I only when B(I,J) is odd:
//       O_I <- cos(theta) O_I + (-1)^{(B(I,J)+1)/2} sin(theta) O_{I xor J}
//    (Eq. update_rule).  The sign is taken from B of the RECEIVING index I,
//    as in Eq. update_rule (reading: Appendix A's list tuple writes the same
//    rule with the source index; the equation is the one that reproduces the
//    exact Heisenberg evolution).
//  * Truncation after every gate: drop I when |O_I| <= eps0 * max_I |O_I|,
//    the max taken over the whole operator after the gate (Eq. truncation1).
//    eps0 <= 0 keeps every generated string, exact zeros included.
//  * Angles within 1e-12*max(1,|theta|) of k*pi/2 use exact (cos, sin) in
//    {0, +-1}; a zero factor is a structural absence (no string is created
//    for it).
//  * <Z> = sum of O_I over strings made of id and sigma_z only, because
//    <0|sigma_I|0> = 1 for those and 0 otherwise (Eq. magnetization).
//  * Several coefficient lanes per string: a lane is an independent operator
//    (its own initial coefficients and angles) sharing the key set; a string
//    exists when any lane created it, and truncation keeps a string when any
//    lane a has |O_I,a| > eps0 * max_I |O_I,a|.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC

#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

namespace {

using Key = std::array<uint64_t, 4>;  // 256-bit multi-index, qubit i at bits 2i (low), 2i+1 (high)

inline int code_of(const Key& I, int q) {
    const int bit = 2 * q;
    return int((I[bit >> 6] >> (bit & 63)) & 3u);
}

// Levi-Civita symbol eps_{ijk} on {1,2,3}.
inline int levi_civita(int i, int j, int k) {
    if (i == j || j == k || i == k) return 0;
    // cyclic permutations of (1,2,3) are +1
    if ((i == 1 && j == 2 && k == 3) || (i == 2 && j == 3 && k == 1) || (i == 3 && j == 1 && k == 2))
        return 1;
    return -1;
}

// Local phase b(I_i, J_i) of Eq. orqaproduct.
inline int local_b(int a, int c) {
    if (a == 0 || c == 0) return 0;
    int s = 0;
    for (int k = 1; k <= 3; ++k) s += levi_civita(a, c, k);
    return s;
}

struct Gate {
    Key J;
    std::vector<int> support;   // qubits where J_i != 00 (b vanishes elsewhere)
    std::vector<double> cs, sn;  // per lane
};

// Exact trigonometry at Clifford angles, libm otherwise.
void classify(double theta, double* c, double* s) {
    const double half_pi = M_PI / 2.0;
    const double k = std::nearbyint(theta / half_pi);
    if (std::fabs(theta - k * half_pi) <= 1e-12 * std::fmax(1.0, std::fabs(theta))) {
        long m = long(k) % 4;
        if (m < 0) m += 4;
        static const double C[4] = {1.0, 0.0, -1.0, 0.0};
        static const double S[4] = {0.0, 1.0, 0.0, -1.0};
        *c = C[m];
        *s = S[m];
        return;
    }
    *c = std::cos(theta);
    *s = std::sin(theta);
}

// Input words (x0,x1,z0,z1), qubit q at word q>>6 bit q&63  ->  2-bit codes.
// Code (h,l) with value 2h+l: sigma_x=01, sigma_y=10, sigma_z=11, so
// h = z and l = x xor z.
Key key_from_xz(const uint64_t* w, int nq) {
    Key I{0, 0, 0, 0};
    for (int q = 0; q < nq; ++q) {
        const uint64_t x = (w[q >> 6] >> (q & 63)) & 1u;
        const uint64_t z = (w[2 + (q >> 6)] >> (q & 63)) & 1u;
        const uint64_t h = z, l = x ^ z;
        const int bit = 2 * q;
        I[bit >> 6] |= ((h << 1) | l) << (bit & 63);
    }
    return I;
}

void xz_from_key(const Key& I, int nq, uint64_t* w) {
    w[0] = w[1] = w[2] = w[3] = 0;
    for (int q = 0; q < nq; ++q) {
        const int c = code_of(I, q);
        const uint64_t h = uint64_t(c >> 1), l = uint64_t(c & 1);
        const uint64_t x = h ^ l, z = h;
        w[q >> 6] |= x << (q & 63);
        w[2 + (q >> 6)] |= z << (q & 63);
    }
}

template <int MAXL>
struct Operator {
    using Coef = std::array<double, MAXL>;
    int nq = 0, L = 1;
    std::map<Key, Coef> O;
    double updates = 0.0;  // sum over gates of |O| before the gate

    int B(const Key& I, const Gate& g) const {
        int s = 0;
        for (int q : g.support) s += local_b(code_of(I, q), code_of(g.J, q));
        return s;
    }

    // (-1)^{(B+1)/2} for odd B (B may be negative).
    static double sign_of(int b) {
        const int e = (b + 1) / 2;  // exact: b odd
        return (e % 2 == 0) ? 1.0 : -1.0;
    }

    void apply(const Gate& g) {
        updates += double(O.size());
        bool any_c = false, any_s = false;
        for (int a = 0; a < L; ++a) {
            any_c |= (g.cs[a] != 0.0);
            any_s |= (g.sn[a] != 0.0);
        }
        std::map<Key, Coef> next;
        for (const auto& kv : O) {
            const Key& I = kv.first;
            const Coef& c = kv.second;
            const int phi = B(I, g);
            if (phi % 2 == 0) {  // commuting: O_I unchanged
                Coef& dst = slot(next, I);
                for (int a = 0; a < L; ++a) dst[a] += c[a];
                continue;
            }
            if (any_c) {  // cos(theta) O_I stays at I
                Coef& dst = slot(next, I);
                for (int a = 0; a < L; ++a)
                    if (g.cs[a] != 0.0) dst[a] += g.cs[a] * c[a];
            }
            if (any_s) {  // sin(theta) O_I is received by K = I xor J
                Key K;
                for (int w = 0; w < 4; ++w) K[w] = I[w] ^ g.J[w];
                const double s = sign_of(B(K, g));
                Coef& dst = slot(next, K);
                for (int a = 0; a < L; ++a)
                    if (g.sn[a] != 0.0) dst[a] += (s * g.sn[a]) * c[a];
            }
        }
        O.swap(next);
    }

    static Coef& slot(std::map<Key, Coef>& m, const Key& k) {
        auto it = m.find(k);
        if (it == m.end()) {
            Coef z;
            z.fill(0.0);
            it = m.emplace(k, z).first;
        }
        return it->second;
    }

    void truncate(double eps0) {
        if (!(eps0 > 0.0)) return;
        std::array<double, MAXL> M;
        M.fill(0.0);
        for (const auto& kv : O)
            for (int a = 0; a < L; ++a) M[a] = std::fmax(M[a], std::fabs(kv.second[a]));
        std::array<double, MAXL> thr;
        for (int a = 0; a < L; ++a) thr[a] = eps0 * M[a];
        for (auto it = O.begin(); it != O.end();) {
            bool keep = false;
            for (int a = 0; a < L; ++a) keep |= (std::fabs(it->second[a]) > thr[a]);
            if (keep) ++it;
            else it = O.erase(it);
        }
    }

    bool xz_free(const Key& I) const {
        for (int q = 0; q < nq; ++q) {
            const int c = code_of(I, q);
            if (c == 1 || c == 2) return false;
        }
        return true;
    }
};

struct State {
    int nq = 0, L = 1;
    Operator<1>* op1 = nullptr;
    Operator<32>* opL = nullptr;
};

template <class F>
auto with_op(State* s, F&& f) {
    if (s->op1) return f(*s->op1);
    return f(*s->opL);
}

}  // namespace

extern "C" {

typedef struct State orc_state;

// terms: n_terms x 4 words (x0,x1,z0,z1); coeffs: n_terms x n_lanes.
int orc_create(int n_qubits, int n_lanes, const uint64_t* terms, const double* coeffs,
               size_t n_terms, orc_state** out) {
    if (n_qubits < 1 || n_qubits > 128 || n_lanes < 1 || n_lanes > 32 || !out) return -1;
    State* s = new State;
    s->nq = n_qubits;
    s->L = n_lanes;
    if (n_lanes == 1) s->op1 = new Operator<1>;
    else s->opL = new Operator<32>;
    with_op(s, [&](auto& op) {
        op.nq = n_qubits;
        op.L = n_lanes;
        for (size_t t = 0; t < n_terms; ++t) {
            const Key I = key_from_xz(terms + 4 * t, n_qubits);
            auto& dst = op.slot(op.O, I);
            for (int a = 0; a < n_lanes; ++a) dst[a] += coeffs[t * n_lanes + a];
        }
        return 0;
    });
    *out = s;
    return 0;
}

void orc_destroy(orc_state* s) {
    if (!s) return;
    delete s->op1;
    delete s->opL;
    delete s;
}

// gens: n_gates x 4 words; thetas: n_gates x n_lanes.  Gates run in the order
// given (Heisenberg order).  eps0 > 0 truncates after every gate.
int orc_apply(orc_state* s, const uint64_t* gens, const double* thetas, size_t n_gates, double eps0) {
    if (!s) return -1;
    for (size_t g = 0; g < n_gates; ++g) {
        Gate G;
        G.J = key_from_xz(gens + 4 * g, s->nq);
        for (int q = 0; q < s->nq; ++q)
            if (code_of(G.J, q) != 0) G.support.push_back(q);
        G.cs.resize(s->L);
        G.sn.resize(s->L);
        for (int a = 0; a < s->L; ++a) classify(thetas[g * s->L + a], &G.cs[a], &G.sn[a]);
        with_op(s, [&](auto& op) {
            op.apply(G);
            op.truncate(eps0);
            return 0;
        });
    }
    return 0;
}

int orc_truncate(orc_state* s, double eps0) {
    if (!s) return -1;
    return with_op(s, [&](auto& op) {
        op.truncate(eps0);
        return 0;
    });
}

size_t orc_size(orc_state* s) {
    return with_op(s, [&](auto& op) { return op.O.size(); });
}

double orc_updates(orc_state* s) {
    return with_op(s, [&](auto& op) { return op.updates; });
}

// <Z> per lane: coefficients of id/sigma_z-only strings, summed in key order.
int orc_expectation_z(orc_state* s, double* out) {
    return with_op(s, [&](auto& op) {
        for (int a = 0; a < op.L; ++a) out[a] = 0.0;
        for (const auto& kv : op.O)
            if (op.xz_free(kv.first))
                for (int a = 0; a < op.L; ++a) out[a] += kv.second[a];
        return 0;
    });
}

int orc_norm2(orc_state* s, double* out) {
    return with_op(s, [&](auto& op) {
        for (int a = 0; a < op.L; ++a) out[a] = 0.0;
        for (const auto& kv : op.O)
            for (int a = 0; a < op.L; ++a) out[a] += kv.second[a] * kv.second[a];
        return 0;
    });
}

// Export up to `cap` strings as (x0,x1,z0,z1) words + lane coefficients, in
// the oracle's own key order.  Returns the number written.
size_t orc_export(orc_state* s, uint64_t* terms, double* coeffs, size_t cap) {
    return with_op(s, [&](auto& op) {
        size_t i = 0;
        for (const auto& kv : op.O) {
            if (i >= cap) break;
            xz_from_key(kv.first, op.nq, terms + 4 * i);
            for (int a = 0; a < op.L; ++a) coeffs[i * op.L + a] = kv.second[a];
            ++i;
        }
        return i;
    });
}

// Phase exponent B(I,J) of Eq. orqaproduct for two strings given as x/z words
// (exposed for the algebra checks).
int orc_phase_B(int n_qubits, const uint64_t* I_xz, const uint64_t* J_xz) {
    const Key I = key_from_xz(I_xz, n_qubits), J = key_from_xz(J_xz, n_qubits);
    int s = 0;
    for (int q = 0; q < n_qubits; ++q) s += local_b(code_of(I, q), code_of(J, q));
    return s;
}

}  // extern "C"
