// Netlist builders of the k-bit two's-complement operators (§3.3, §4.3-4.5,
// Algs. 3-6), of one fixed-point gradient-descent step of linear regression
// (§4.6), of the closed-form regression (§3.4 Eqs. (2)-(3), Alg. 7) and of
// Table 2's NAND-only gates.
//
// Wire 0 / wire 1 are the constants 0 / 1, inputs come next, every gate adds
// one wire.  Adder: ripple of one-bit adders x = a^b, s = x^c,
// c' = (a&b)|(x&c) with carry-in 0 (5k gates, §5.2).  Subtractor: k
// bootstrapped XORs with 1, then the adder with carry-in 1 (6k, §5.4).
// Multiplier: signed Baugh-Wooley carry-save array (AND partial products,
// NAND where exactly one operand bit has negative weight, full/half adders
// per row, a final ripple adder, constants 2^k and 2^(2k-1)).  Divider:
// compensation to absolute values, a non-restoring array of CAS cells
// (out = a^((b^p)^c), c' = ((a|c)&(b^p))|(a&c)), remainder correction and
// compensation back to signed quotient and remainder.  Multiplier, divider
// and the regression step fold gates with constant inputs.
#include <algorithm>
#include <map>
#include <vector>

#include "mk_internal.h"

namespace mk {
namespace {

constexpr int kZero = 0, kOne = 1;

class Builder {
  public:
    explicit Builder(bool fold) : fold_(fold) {}
    int wires = 2;
    std::vector<mk_gate> gates;
    std::vector<int> inputs, outputs;

    int input() {
        inputs.push_back(wires);
        return wires++;
    }
    int emit(int t, int a, int b) {
        gates.push_back(mk_gate{t, a, b, wires});
        return wires++;
    }
    int inv(int a) {
        if (fold_) {
            if (a == kZero || a == kOne) return 1 - a;
            auto it = inverse_.find(a);
            if (it != inverse_.end()) return it->second;
        }
        const int w = emit(MK_GATE_NOT, a, 0);
        inverse_[w] = a;
        return w;
    }
    int g(int t, int a, int b) {
        if (fold_) {
            const bool ca = a <= kOne, cb = b <= kOne;
            if (ca && cb) return eval(t, a, b);
            if (ca) std::swap(a, b);
            if (ca || cb) {
                const int v = b;  // a is a wire, b a constant
                switch (t) {
                    case MK_GATE_AND: return v ? a : kZero;
                    case MK_GATE_OR: return v ? kOne : a;
                    case MK_GATE_XOR: return v ? inv(a) : a;
                    case MK_GATE_XNOR: return v ? a : inv(a);
                    case MK_GATE_NAND: return v ? inv(a) : kOne;
                    case MK_GATE_NOR: return v ? kZero : inv(a);
                }
            }
        }
        return emit(t, a, b);
    }
    static int eval(int t, int a, int b) {
        switch (t) {
            case MK_GATE_NAND: return 1 - (a & b);
            case MK_GATE_AND: return a & b;
            case MK_GATE_OR: return a | b;
            case MK_GATE_NOR: return 1 - (a | b);
            case MK_GATE_XOR: return a ^ b;
            default: return 1 - (a ^ b);
        }
    }
    // one-bit adder: 5 gates
    void fa(int a, int b, int c, int &s, int &co) {
        const int x = g(MK_GATE_XOR, a, b);
        s = g(MK_GATE_XOR, x, c);
        const int t1 = g(MK_GATE_AND, a, b);
        const int t2 = g(MK_GATE_AND, x, c);
        co = g(MK_GATE_OR, t1, t2);
    }
    // sum of 1..3 equally weighted bits; co = -1 when no carry is formed
    void sum_bits(const std::vector<int> &bits, bool want_carry, int &s, int &co) {
        co = -1;
        if (bits.size() == 1) {
            s = bits[0];
        } else if (bits.size() == 2) {
            s = g(MK_GATE_XOR, bits[0], bits[1]);
            if (want_carry) co = g(MK_GATE_AND, bits[0], bits[1]);
        } else if (want_carry) {
            fa(bits[0], bits[1], bits[2], s, co);
        } else {
            s = g(MK_GATE_XOR, g(MK_GATE_XOR, bits[0], bits[1]), bits[2]);
        }
    }
    std::vector<int> ripple(const std::vector<int> &a, const std::vector<int> &b, int cin) {
        std::vector<int> out(a.size());
        int c = cin;
        for (size_t i = 0; i < a.size(); ++i) fa(a[i], b[i], c, out[i], c);
        return out;
    }
    // (x XOR s) + s
    std::vector<int> compensate(const std::vector<int> &x, int s) {
        std::vector<int> y(x.size()), out(x.size());
        for (size_t i = 0; i < x.size(); ++i) y[i] = g(MK_GATE_XOR, x[i], s);
        int c = s;
        for (size_t i = 0; i < y.size(); ++i) {
            out[i] = g(MK_GATE_XOR, y[i], c);
            if (i + 1 < y.size()) c = g(MK_GATE_AND, y[i], c);
        }
        return out;
    }
    std::vector<int> multiply(const std::vector<int> &a, const std::vector<int> &b) {
        const int k = (int)a.size();
        std::vector<std::vector<int>> q(k, std::vector<int>(k));
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j)
                q[i][j] = g(((i == k - 1) != (j == k - 1)) ? MK_GATE_NAND : MK_GATE_AND, a[j], b[i]);
        std::map<int, int> S, C;
        for (int w = 0; w < k; ++w) S[w] = q[0][w];
        std::vector<int> out;
        out.push_back(S[0]);
        S.erase(0);
        for (int i = 1; i < k; ++i) {
            std::map<int, int> S2, C2;
            for (int w = i; w < i + k; ++w) {
                std::vector<int> bits;
                if (S.count(w)) bits.push_back(S[w]);
                if (C.count(w)) bits.push_back(C[w]);
                bits.push_back(q[i][w - i]);
                if (i == 1 && w == k) bits.push_back(kOne);
                int s, co;
                sum_bits(bits, true, s, co);
                S2[w] = s;
                if (co >= 0) C2[w + 1] = co;
            }
            S.swap(S2);
            C.swap(C2);
            out.push_back(S[i]);
            S.erase(i);
        }
        int c = -1;
        for (int w = k; w < 2 * k; ++w) {
            std::vector<int> bits;
            if (S.count(w)) bits.push_back(S[w]);
            if (C.count(w)) bits.push_back(C[w]);
            if (c >= 0) bits.push_back(c);
            int s;
            sum_bits(bits, w < 2 * k - 1, s, c);
            out.push_back(s);
        }
        out[2 * k - 1] = inv(out[2 * k - 1]);
        return out;
    }
    void cas(int a, int b, int c, int p, int &o, int &co) {
        const int t = g(MK_GATE_XOR, b, p);
        const int u = g(MK_GATE_XOR, t, c);
        o = g(MK_GATE_XOR, a, u);
        const int x = g(MK_GATE_AND, g(MK_GATE_OR, a, c), t);
        co = g(MK_GATE_OR, x, g(MK_GATE_AND, a, c));
    }
    void divide(const std::vector<int> &A, const std::vector<int> &B, std::vector<int> &quot,
                std::vector<int> &rem) {
        const int kA = (int)A.size(), k = (int)B.size();
        const int sA = A[kA - 1], sB = B[k - 1];
        const std::vector<int> ua = compensate(A, sA);
        std::vector<int> D = compensate(B, sB);
        D.push_back(kZero);
        std::vector<int> R(k + 1, kZero), q;
        int p = kOne;
        for (int i = kA - 1; i >= 0; --i) {
            std::vector<int> Rs(k + 1);
            Rs[0] = ua[i];
            for (int t = 1; t <= k; ++t) Rs[t] = R[t - 1];
            int c = p;
            for (int t = 0; t <= k; ++t) cas(Rs[t], D[t], c, p, R[t], c);
            const int qi = inv(R[k]);
            q.push_back(qi);
            p = qi;
        }
        std::reverse(q.begin(), q.end());
        std::vector<int> corr(k), low(R.begin(), R.begin() + k);
        for (int t = 0; t < k; ++t) corr[t] = g(MK_GATE_AND, D[t], R[k]);
        std::vector<int> r = ripple(low, corr, kZero);
        const int sQ = g(MK_GATE_XOR, sA, sB);
        quot = compensate(std::vector<int>(q.begin(), q.begin() + k), sQ);
        rem = compensate(r, sA);
    }

  private:
    bool fold_;
    std::map<int, int> inverse_;
};

std::vector<int> inputs_n(Builder &b, int n) {
    std::vector<int> v(n);
    for (int i = 0; i < n; ++i) v[i] = b.input();
    return v;
}

int export_netlist(const Builder &b, mk_gate *gates, int32_t *n_gates, int32_t *n_wires,
                   int32_t *inputs, int32_t *outputs) {
    if (gates) {
        if (!inputs || !outputs) return fail(MK_EINVAL, "netlist builder: null output array");
        std::copy(b.gates.begin(), b.gates.end(), gates);
        std::copy(b.inputs.begin(), b.inputs.end(), inputs);
        std::copy(b.outputs.begin(), b.outputs.end(), outputs);
    }
    *n_gates = (int32_t)b.gates.size();
    *n_wires = b.wires;
    return MK_OK;
}

}  // namespace
}  // namespace mk

using namespace mk;

extern "C" {

int mk_build_operator(int op, int kbits, mk_gate *gates, int32_t *n_gates, int32_t *n_wires,
                      int32_t *inputs, int32_t *outputs) {
    if (!n_gates || !n_wires) return fail(MK_EINVAL, "mk_build_operator: null count pointer");
    if (kbits < 1 || kbits > 64) return fail(MK_EINVAL, "mk_build_operator: kbits out of range");
    if ((op == MK_OP_MUL || op >= MK_OP_DIV) && kbits < 2)
        return fail(MK_EINVAL, "mk_build_operator: multiplier and divider need kbits >= 2");
    Builder b(op == MK_OP_MUL || op == MK_OP_DIV || op == MK_OP_DIV2);
    std::vector<int> a = inputs_n(b, op == MK_OP_DIV2 ? 2 * kbits : kbits);
    std::vector<int> c = inputs_n(b, kbits);
    switch (op) {
        case MK_OP_ADD:
            b.outputs = b.ripple(a, c, kZero);
            break;
        case MK_OP_SUB: {
            std::vector<int> nc(kbits);
            for (int i = 0; i < kbits; ++i) nc[i] = b.g(MK_GATE_XOR, c[i], kOne);
            b.outputs = b.ripple(a, nc, kOne);
            break;
        }
        case MK_OP_MUL:
            b.outputs = b.multiply(a, c);
            break;
        case MK_OP_DIV:
        case MK_OP_DIV2: {
            std::vector<int> q, r;
            b.divide(a, c, q, r);
            b.outputs = q;
            b.outputs.insert(b.outputs.end(), r.begin(), r.end());
            break;
        }
        default:
            return fail(MK_EINVAL, "mk_build_operator: unknown operator");
    }
    return export_netlist(b, gates, n_gates, n_wires, inputs, outputs);
}

int mk_build_naive_gate(int type, mk_gate *gates, int32_t *n_gates, int32_t *n_wires, int32_t *inputs,
                        int32_t *outputs) {
    if (!n_gates || !n_wires) return fail(MK_EINVAL, "mk_build_naive_gate: null count pointer");
    if (type < 0 || type > MK_GATE_NOT) return fail(MK_EINVAL, "mk_build_naive_gate: unknown gate type");
    Builder b(false);  // no folding: NAND(x, x) stays a bootstrapped gate
    std::vector<int> in = inputs_n(b, 2);
    const int x = in[0], y = in[1];
    auto nand = [&](int u, int v) { return b.g(MK_GATE_NAND, u, v); };
    auto naive_or = [&](int u, int v) {
        const int nu = nand(u, u);  // sequenced: the gate order is the netlist
        const int nv = nand(v, v);
        return nand(nu, nv);
    };
    auto naive_xor = [&](int u, int v) {
        const int n = nand(u, v);
        const int p = nand(u, n);
        const int q = nand(v, n);
        return nand(p, q);
    };
    int out;
    switch (type) {
        case MK_GATE_NAND: out = nand(x, y); break;
        case MK_GATE_AND: {
            const int n = nand(x, y);
            out = nand(n, n);
            break;
        }
        case MK_GATE_OR: out = naive_or(x, y); break;
        case MK_GATE_NOR: {
            const int o = naive_or(x, y);
            out = nand(o, o);
            break;
        }
        case MK_GATE_XOR: out = naive_xor(x, y); break;
        case MK_GATE_XNOR: {
            const int z = naive_xor(x, y);
            out = nand(z, z);
            break;
        }
        default: out = nand(x, x); break;  // NOT
    }
    b.outputs = {out};
    return export_netlist(b, gates, n_gates, n_wires, inputs, outputs);
}

int mk_build_lr_step(int m, int d, int shift, mk_gate *gates, int32_t *n_gates, int32_t *n_wires,
                     int32_t *inputs, int32_t *outputs) {
    if (!n_gates || !n_wires) return fail(MK_EINVAL, "mk_build_lr_step: null count pointer");
    if (m < 1 || d < 1 || shift < 0 || shift > 15 || (size_t)m * d > 4096)
        return fail(MK_EINVAL, "mk_build_lr_step: size out of range");
    constexpr int kB = 16, kF = 8;
    Builder b(true);
    std::vector<std::vector<std::vector<int>>> X(m, std::vector<std::vector<int>>(d));
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < d; ++j) X[i][j] = inputs_n(b, kB);
    std::vector<std::vector<int>> y(m), w(d);
    for (int i = 0; i < m; ++i) y[i] = inputs_n(b, kB);
    for (int j = 0; j < d; ++j) w[j] = inputs_n(b, kB);
    auto mq = [&](const std::vector<int> &x, const std::vector<int> &z) {
        std::vector<int> p = b.multiply(x, z);
        return std::vector<int>(p.begin() + kF, p.begin() + kF + kB);
    };
    auto sub = [&](const std::vector<int> &x, const std::vector<int> &z) {
        std::vector<int> nz(kB);
        for (int i = 0; i < kB; ++i) nz[i] = b.g(MK_GATE_XOR, z[i], kOne);
        return b.ripple(x, nz, kOne);
    };
    std::vector<std::vector<int>> r(m);
    for (int i = 0; i < m; ++i) {
        std::vector<int> acc = mq(X[i][0], w[0]);
        for (int j = 1; j < d; ++j) acc = b.ripple(acc, mq(X[i][j], w[j]), kZero);
        r[i] = sub(acc, y[i]);
    }
    for (int j = 0; j < d; ++j) {
        std::vector<int> acc = mq(X[0][j], r[0]);
        for (int i = 1; i < m; ++i) acc = b.ripple(acc, mq(X[i][j], r[i]), kZero);
        std::vector<int> step(kB);
        for (int t = 0; t < kB; ++t) step[t] = acc[std::min(t + shift, kB - 1)];
        std::vector<int> nw = sub(w[j], step);
        b.outputs.insert(b.outputs.end(), nw.begin(), nw.end());
    }
    return export_netlist(b, gates, n_gates, n_wires, inputs, outputs);
}

int mk_build_lr_formula(int m, int frac, mk_gate *gates, int32_t *n_gates, int32_t *n_wires,
                        int32_t *inputs, int32_t *outputs) {
    if (!n_gates || !n_wires) return fail(MK_EINVAL, "mk_build_lr_formula: null count pointer");
    if (m < 1 || m > 4096 || frac < 0 || frac > 15)
        return fail(MK_EINVAL, "mk_build_lr_formula: size out of range");
    constexpr int kIn = 8, kW = 16;
    Builder b(true);
    std::vector<std::vector<int>> x(m), y(m);
    for (int i = 0; i < m; ++i) x[i] = inputs_n(b, kIn);
    for (int i = 0; i < m; ++i) y[i] = inputs_n(b, kIn);
    std::vector<int> cm(kW);
    for (int t = 0; t < kW; ++t) cm[t] = (m >> t) & 1 ? kOne : kZero;
    // v sign-extended to `bits`, optionally times 2^frac (wiring only)
    auto widen = [&](const std::vector<int> &v, int bits, int shift) {
        std::vector<int> o(shift, kZero);
        o.insert(o.end(), v.begin(), v.end());
        o.resize(bits, v.back());
        return o;
    };
    auto sub = [&](const std::vector<int> &u, const std::vector<int> &v) {
        std::vector<int> nv(v.size());
        for (size_t i = 0; i < v.size(); ++i) nv[i] = b.g(MK_GATE_XOR, v[i], kOne);
        return b.ripple(u, nv, kOne);
    };
    auto total = [&](const std::vector<std::vector<int>> &terms) {
        std::vector<int> acc = terms[0];
        for (size_t i = 1; i < terms.size(); ++i) acc = b.ripple(acc, terms[i], kZero);
        return acc;
    };
    auto quotient = [&](const std::vector<int> &num, const std::vector<int> &den) {
        std::vector<int> q, r;
        b.divide(num, den, q, r);
        return q;
    };
    std::vector<std::vector<int>> ex(m), ey(m);
    for (int i = 0; i < m; ++i) ex[i] = widen(x[i], kW, 0);
    for (int i = 0; i < m; ++i) ey[i] = widen(y[i], kW, 0);
    const std::vector<int> sx = total(ex), sy = total(ey);
    std::vector<int> xbar = quotient(sx, cm), ybar = quotient(sy, cm);
    xbar.resize(kIn);
    ybar.resize(kIn);
    std::vector<std::vector<int>> dx(m), dy(m), pn(m), pd(m);
    for (int i = 0; i < m; ++i) dx[i] = sub(x[i], xbar);
    for (int i = 0; i < m; ++i) dy[i] = sub(y[i], ybar);
    for (int i = 0; i < m; ++i) pn[i] = b.multiply(dy[i], dx[i]);
    const std::vector<int> num = total(pn);
    for (int i = 0; i < m; ++i) pd[i] = b.multiply(dx[i], dx[i]);
    const std::vector<int> den = total(pd);
    const std::vector<int> omega = quotient(widen(num, 2 * kW, frac), den);
    const std::vector<int> prod = b.multiply(omega, sx);
    const std::vector<int> u = sub(widen(sy, 2 * kW, frac), prod);
    const std::vector<int> icpt = quotient(u, cm);
    b.outputs = omega;
    b.outputs.insert(b.outputs.end(), icpt.begin(), icpt.end());
    return export_netlist(b, gates, n_gates, n_wires, inputs, outputs);
}

}  // extern "C"
