// Givens stages of the generated A = Q Sigma G^T (eq. (16), section 4) as
// seen from one index: which rotation of stage t touches index i, its
// partner, its angle and whether i is the first or second element.
//
// Stage t (1-based) of a side with bijection pi pairs positions
// (2k, 2k+1) for odd t and (2k+1, 2k+2 mod N) for even t (the adjacent and
// shifted stages of section 4.2, under a random permutation as in 4.1).
// The rotation on pair (f, g) is G(f, g, theta): (z_f, z_g) ->
// (c z_f - s z_g, s z_f + c z_g) (section 4, display of G(i, j, theta)).
#pragma once

#include "common.hpp"

namespace l1ls {

struct PairRef {
    int32_t partner;
    bool first;
    double c, s;
};

__device__ __forceinline__ PairRef pair_of(const SideTables& T, int t, int32_t i) {
    const int64_t N = T.N;
    const int64_t a = T.pinv[i];
    int64_t k, mate;
    bool first;
    if (t & 1) {
        k = a >> 1;
        first = (a & 1) == 0;
        mate = a ^ 1;
    } else if (a & 1) {
        k = a >> 1;
        first = true;
        mate = (a + 1 == N) ? 0 : a + 1;
    } else {
        first = false;
        k = (a == 0) ? (N / 2 - 1) : (a / 2 - 1);
        mate = (a == 0) ? (N - 1) : (a - 1);
    }
    const double* cs = T.cs[t - 1];
    PairRef p;
    p.partner = T.perm[mate];
    p.first = first;
    p.c = cs[2 * k];
    p.s = cs[2 * k + 1];
    return p;
}

// Coefficient of z_i in the partner's output: G(f,g) column f is (c, s),
// column g is (-s, c); the transpose swaps the off-diagonal signs.
__device__ __forceinline__ double partner_coef(const PairRef& p, bool transpose) {
    const bool plus = (p.first != transpose);
    return plus ? p.s : -p.s;
}

// One stage applied to a whole vector, out-of-place (out != in).
// Element i of the output uses the two inputs of its pair in the order of
// the rotation formula, with round-to-nearest intrinsics (no contraction).
template <typename T>
__device__ __forceinline__ T stage_elem(const PairRef& p, T zi, T zp, bool transpose);

template <>
__device__ __forceinline__ double stage_elem<double>(const PairRef& p, double zi, double zp, bool transpose) {
    // forward, i first:  c z_i - s z_p;  i second: s z_p + c z_i
    // transpose, i first: c z_i + s z_p; i second: -s z_p + c z_i
    if (p.first) {
        const double a = __dmul_rn(p.c, zi), b = __dmul_rn(p.s, zp);
        return transpose ? __dadd_rn(a, b) : __dsub_rn(a, b);
    }
    const double a = __dmul_rn(transpose ? -p.s : p.s, zp), b = __dmul_rn(p.c, zi);
    return __dadd_rn(a, b);
}

template <>
__device__ __forceinline__ float stage_elem<float>(const PairRef& p, float zi, float zp, bool transpose) {
    const float c = (float)p.c, s = (float)p.s;
    if (p.first) {
        const float a = __fmul_rn(c, zi), b = __fmul_rn(s, zp);
        return transpose ? __fadd_rn(a, b) : __fsub_rn(a, b);
    }
    const float a = __fmul_rn(transpose ? -s : s, zp), b = __fmul_rn(c, zi);
    return __fadd_rn(a, b);
}

// Small sparse vector (index, value) kept in registers.
template <int MAXE>
struct SparseVec {
    int cnt;
    int32_t idx[MAXE];
    double val[MAXE];
    __device__ __forceinline__ void add(int32_t i, double v) {
        for (int e = 0; e < cnt; ++e)
            if (idx[e] == i) {
                val[e] = __dadd_rn(val[e], v);
                return;
            }
        if (cnt < MAXE) {
            idx[cnt] = i;
            val[cnt] = v;
            ++cnt;
        }
    }
};

// out = S_t v (transpose: S_t^T v) for a sparse v.
template <int MAXE>
__device__ __forceinline__ void stage_sparse(const SideTables& T, int t, bool transpose,
                                             const SparseVec<MAXE>& v, SparseVec<MAXE>& out) {
    out.cnt = 0;
    for (int e = 0; e < v.cnt; ++e) {
        const PairRef p = pair_of(T, t, v.idx[e]);
        out.add(v.idx[e], __dmul_rn(p.c, v.val[e]));
        out.add(p.partner, __dmul_rn(partner_coef(p, transpose), v.val[e]));
    }
}

template <int MAXE>
__device__ __forceinline__ void sort_sparse(SparseVec<MAXE>& v) {
    for (int a = 1; a < v.cnt; ++a) {
        const int32_t ki = v.idx[a];
        const double kv = v.val[a];
        int b = a - 1;
        while (b >= 0 && v.idx[b] > ki) {
            v.idx[b + 1] = v.idx[b];
            v.val[b + 1] = v.val[b];
            --b;
        }
        v.idx[b + 1] = ki;
        v.val[b + 1] = kv;
    }
}

// Column j of A = Q Sigma G^T: e_j through G^T (stage r first), Sigma,
// then Q (stage 1 first).  Result sorted by row.
template <int MAXE>
__device__ __forceinline__ void column_of_A(const SideTables& Gs, const SideTables& Qs, int rounds,
                                            const double* sigma, int32_t j, SparseVec<MAXE>& out) {
    SparseVec<MAXE> a, b;
    a.cnt = 1;
    a.idx[0] = j;
    a.val[0] = 1.0;
    SparseVec<MAXE>* cur = &a;
    SparseVec<MAXE>* nxt = &b;
    for (int t = rounds; t >= 1; --t) {
        stage_sparse(Gs, t, true, *cur, *nxt);
        SparseVec<MAXE>* tmp = cur; cur = nxt; nxt = tmp;
    }
    for (int e = 0; e < cur->cnt; ++e) cur->val[e] = __dmul_rn(sigma[cur->idx[e]], cur->val[e]);
    for (int t = 1; t <= rounds; ++t) {
        stage_sparse(Qs, t, false, *cur, *nxt);
        SparseVec<MAXE>* tmp = cur; cur = nxt; nxt = tmp;
    }
    out = *cur;
    sort_sparse(out);
}

// Row i of A as A^T e_i = G Sigma^T Q^T e_i: Q^T (stage r first), drop
// indices >= n, Sigma, then G (stage 1 first).  Only the column set is
// used (values are taken from the stored columns).  Sorted by column.
template <int MAXE>
__device__ __forceinline__ void row_pattern_of_A(const SideTables& Gs, const SideTables& Qs, int rounds,
                                                 int64_t n, const double* sigma, int32_t i,
                                                 SparseVec<MAXE>& out) {
    SparseVec<MAXE> a, b;
    a.cnt = 1;
    a.idx[0] = i;
    a.val[0] = 1.0;
    SparseVec<MAXE>* cur = &a;
    SparseVec<MAXE>* nxt = &b;
    for (int t = rounds; t >= 1; --t) {
        stage_sparse(Qs, t, true, *cur, *nxt);
        SparseVec<MAXE>* tmp = cur; cur = nxt; nxt = tmp;
    }
    int keep = 0;
    for (int e = 0; e < cur->cnt; ++e)
        if (cur->idx[e] < n) {
            cur->idx[keep] = cur->idx[e];
            cur->val[keep] = __dmul_rn(sigma[cur->idx[e]], cur->val[e]);
            ++keep;
        }
    cur->cnt = keep;
    for (int t = 1; t <= rounds; ++t) {
        stage_sparse(Gs, t, false, *cur, *nxt);
        SparseVec<MAXE>* tmp = cur; cur = nxt; nxt = tmp;
    }
    out = *cur;
    sort_sparse(out);
}

}  // namespace l1ls
