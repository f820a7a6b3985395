// Host plan builder: validation, multipliers, local tables, channel list, device image.
//
// Mixed-radix indexing (Sec. III): M_k = prod_{l>k} d_l with site 0 most significant, D = prod d_l.
// Off-diagonal terms become channels with a fixed integer offset Delta = q_a M_a + q_b M_b and a
// per-digit coefficient table (Sec. IV, Eq. sourceoffset); diagonal terms (S_z, (S_z)^2, S_z S_z and
// the boson number operator) are kept apart since their source index is the target itself.
#include <cmath>
#include <cstring>
#include <complex>
#include <map>
#include <tuple>

#include "mrmf_internal.h"

using mrmf::DevChan;
using mrmf::DevDiag;
using mrmf::DevSite;

namespace {

int shift_of(int op) {
    switch (op) {
        case MRMF_OP_RAISE: return 1;
        case MRMF_OP_LOWER: return -1;
        case MRMF_OP_RAISE2: return 2;
        case MRMF_OP_LOWER2: return -2;
        default: return 0;
    }
}
int adjoint_op(int op) {
    switch (op) {
        case MRMF_OP_RAISE: return MRMF_OP_LOWER;
        case MRMF_OP_LOWER: return MRMF_OP_RAISE;
        case MRMF_OP_RAISE2: return MRMF_OP_LOWER2;
        case MRMF_OP_LOWER2: return MRMF_OP_RAISE2;
        default: return op;
    }
}

// Hermiticity of every parameter group h_p (Sec. IV.A: h_- = conj(h_+); Eq. pairham:
// conj(J^{ab}) = J^{bar a bar b}).  Terms are keyed by their operator with the two sites in
// ascending order (operators on different sites commute).
bool groups_hermitian(const std::vector<mrmf_term>& terms, int32_t n_params) {
    using Key = std::tuple<int, int, int, int>;
    std::vector<std::map<Key, std::complex<double>>> groups(n_params);
    std::vector<double> scale(n_params, 0.0);
    for (const auto& t : terms) {
        Key k;
        if (t.site_b < 0)
            k = Key(t.site_a, t.op_a, -1, 0);
        else if (t.site_a < t.site_b)
            k = Key(t.site_a, t.op_a, t.site_b, t.op_b);
        else
            k = Key(t.site_b, t.op_b, t.site_a, t.op_a);
        std::complex<double> w(t.w_re, t.w_im);
        groups[t.param][k] += w;
        scale[t.param] = std::max(scale[t.param], std::abs(w));
    }
    for (int p = 0; p < n_params; ++p) {
        const double tol = 1e-13 * std::max(1.0, scale[p]);
        for (const auto& kv : groups[p]) {
            const Key& k = kv.first;
            Key a(std::get<0>(k), adjoint_op(std::get<1>(k)), std::get<2>(k),
                  std::get<2>(k) < 0 ? 0 : adjoint_op(std::get<3>(k)));
            auto it = groups[p].find(a);
            std::complex<double> wa = it == groups[p].end() ? 0.0 : it->second;
            if (std::abs(kv.second - std::conj(wa)) > tol) return false;
        }
    }
    return true;
}

}  // namespace

namespace mrmf {

// <n|O|n - q> of a local operator at target digit n, 0 where the source digit n - q is outside 0..d-1.
// up[n] = <n|R|n-1>, so R^2 at target n is up[n] up[n-1] and L^2 is up[n+1] up[n+2] (App. B).
double local_factor_host(const mrmf_plan_t* p, int site, int op, int n) {
    const int d = p->d[site], tab = p->tab[site];
    const double* val = p->val.data() + tab;
    const double* up = p->up.data() + tab;
    switch (op) {
        case MRMF_OP_Z: return val[n];
        case MRMF_OP_Z2: return val[n] * val[n];
        case MRMF_OP_RAISE: return n >= 1 ? up[n] : 0.0;
        case MRMF_OP_LOWER: return n <= d - 2 ? up[n + 1] : 0.0;
        case MRMF_OP_RAISE2: return n >= 2 ? up[n] * up[n - 1] : 0.0;
        default: return n <= d - 3 ? up[n + 1] * up[n + 2] : 0.0;
    }
}

}  // namespace mrmf

extern "C" {

const char* mrmf_status_string(mrmf_status s) {
    switch (s) {
        case MRMF_OK: return "ok";
        case MRMF_E_INVALID_ARG: return "invalid argument";
        case MRMF_E_OVERFLOW: return "basis dimension overflows the 62-bit index";
        case MRMF_E_NOT_HERMITIAN: return "a parameter group is not Hermitian";
        case MRMF_E_HIP: return "HIP runtime error";
        case MRMF_E_UNSUPPORTED: return "unsupported";
        case MRMF_E_WORKSPACE: return "workspace or scratch too small";
        default: return "unknown status";
    }
}

int32_t mrmf_version(void) { return 10000; }

mrmf_status mrmf_plan_create(int32_t n_sites, const mrmf_site* sites, int32_t n_terms,
                             const mrmf_term* terms, int32_t n_params, uint32_t flags,
                             mrmf_plan* out) {
    if (!out) return MRMF_E_INVALID_ARG;
    *out = nullptr;
    if (n_sites < 1 || n_sites > mrmf::kMaxSites || !sites) return MRMF_E_INVALID_ARG;
    if (n_terms < 0 || (n_terms > 0 && !terms) || n_params < 0) return MRMF_E_INVALID_ARG;
    if (flags & ~MRMF_REQUIRE_HERMITIAN) return MRMF_E_INVALID_ARG;

    auto* p = new (std::nothrow) mrmf_plan_t();
    if (!p) return MRMF_E_INVALID_ARG;
    p->N = n_sites;
    p->n_params = n_params;
    p->flags = flags;
    p->kind.resize(n_sites);
    p->k.resize(n_sites);
    p->d.resize(n_sites);
    p->M.resize(n_sites);
    for (int i = 0; i < n_sites; ++i) {
        const int kind = sites[i].kind, k = sites[i].k;
        if ((kind != MRMF_SPIN && kind != MRMF_BOSON) || k < 1 || k + 1 > mrmf::kMaxDim) {
            delete p;
            return MRMF_E_INVALID_ARG;
        }
        p->kind[i] = kind;
        p->k[i] = k;
        p->d[i] = k + 1;
    }
    // multipliers and D with the single-word bound D < 2^62
    const int64_t limit = int64_t(1) << 62;
    int64_t acc = 1;
    for (int i = n_sites - 1; i >= 0; --i) {
        p->M[i] = acc;
        if (acc > limit / p->d[i]) {
            delete p;
            return MRMF_E_OVERFLOW;
        }
        acc *= p->d[i];
    }
    if (acc >= limit) {
        delete p;
        return MRMF_E_OVERFLOW;
    }
    p->D = acc;

    // terms
    p->terms.assign(terms, terms + n_terms);
    for (int t = 0; t < n_terms; ++t) {
        const mrmf_term& x = terms[t];
        bool ok = x.site_a >= 0 && x.site_a < n_sites && x.op_a >= MRMF_OP_Z && x.op_a <= MRMF_OP_LOWER2 &&
                  x.param >= 0 && x.param < n_params && std::isfinite(x.w_re) && std::isfinite(x.w_im);
        if (ok && x.site_b >= 0) {
            ok = x.site_b < n_sites && x.site_b != x.site_a && x.op_a != MRMF_OP_Z2 && x.op_a <= MRMF_OP_LOWER &&
                 x.op_b >= MRMF_OP_Z && x.op_b <= MRMF_OP_LOWER && x.op_b != MRMF_OP_Z2;
        } else if (ok) {
            ok = x.site_b == -1;
        }
        if (!ok) {
            delete p;
            return MRMF_E_INVALID_ARG;
        }
    }
    p->hermitian = groups_hermitian(p->terms, n_params);
    if ((flags & MRMF_REQUIRE_HERMITIAN) && !p->hermitian) {
        delete p;
        return MRMF_E_NOT_HERMITIAN;
    }

    // local tables: val[n] = m or n; up[n] = <n|R|n-1> = sqrt(n (d - n)) for a spin
    // (= sqrt(s(s+1) - m(m+1)) at source m = n - 1 - s, App. A Lambda), sqrt(n) for a boson (App. C)
    p->tab.resize(n_sites);
    for (int i = 0; i < n_sites; ++i) {
        p->tab[i] = static_cast<int32_t>(p->val.size());
        const int d = p->d[i];
        for (int n = 0; n < d; ++n) {
            if (p->kind[i] == MRMF_SPIN) {
                p->val.push_back(double(n) - 0.5 * double(p->k[i]));
                p->up.push_back(n == 0 ? 0.0 : std::sqrt(double(n) * double(d - n)));
            } else {
                p->val.push_back(double(n));
                p->up.push_back(std::sqrt(double(n)));
            }
        }
    }

    // channels and diagonal terms
    for (int t = 0; t < n_terms; ++t) {
        const mrmf_term& x = terms[t];
        const int qa = shift_of(x.op_a), qb = x.site_b >= 0 ? shift_of(x.op_b) : 0;
        if (qa == 0 && qb == 0) {
            DevDiag g{};
            g.a = x.site_a;
            g.b = x.site_b;
            g.opa = x.op_a;
            g.opb = x.site_b >= 0 ? x.op_b : MRMF_OP_Z;
            g.param = x.param;
            g.term = t;
            g.wr = x.w_re;
            g.wi = x.w_im;
            p->diags.push_back(g);
        } else {
            DevChan c{};
            c.a = x.site_a;
            c.b = x.site_b;
            c.opa = x.op_a;
            c.opb = x.site_b >= 0 ? x.op_b : MRMF_OP_Z;
            c.qa = qa;
            c.qb = qb;
            c.param = x.param;
            c.term = t;
            c.delta = int64_t(qa) * p->M[x.site_a] + (x.site_b >= 0 ? int64_t(qb) * p->M[x.site_b] : 0);
            c.wr = x.w_re;
            c.wi = x.w_im;
            p->chans.push_back(c);
        }
    }

    // default tiling: the low sites whose product stays <= 1024 rows
    {
        int k_in = n_sites;
        int64_t T = 1;
        while (k_in > 0 && T * p->d[k_in - 1] <= 1024) {
            --k_in;
            T *= p->d[k_in];
        }
        p->tiling.k_in = k_in;
        p->tiling.T_in = static_cast<int32_t>(T);
    }

    // device image: [sites][channels][diagonal terms][val][up], sections 256-aligned
    using mrmf::align_up;
    size_t off = 0;
    p->off_site = off;
    off = align_up(off + sizeof(DevSite) * n_sites, 256);
    p->off_chan = off;
    off = align_up(off + sizeof(DevChan) * std::max<size_t>(1, p->chans.size()), 256);
    p->off_diag = off;
    off = align_up(off + sizeof(DevDiag) * std::max<size_t>(1, p->diags.size()), 256);
    p->off_val = off;
    off = align_up(off + sizeof(double) * p->val.size(), 256);
    p->off_up = off;
    off = align_up(off + sizeof(double) * p->up.size(), 256);
    p->ws_bytes = off;
    p->image.assign(off, 0);
    for (int i = 0; i < n_sites; ++i) {
        DevSite s{};
        s.d = p->d[i];
        s.tab = p->tab[i];
        s.kind = p->kind[i];
        s.M = p->M[i];
        s.magic = ~uint64_t(0) / uint64_t(p->d[i]) + 1;
        std::memcpy(p->image.data() + p->off_site + i * sizeof(DevSite), &s, sizeof(s));
    }
    if (!p->chans.empty())
        std::memcpy(p->image.data() + p->off_chan, p->chans.data(), sizeof(DevChan) * p->chans.size());
    if (!p->diags.empty())
        std::memcpy(p->image.data() + p->off_diag, p->diags.data(), sizeof(DevDiag) * p->diags.size());
    std::memcpy(p->image.data() + p->off_val, p->val.data(), sizeof(double) * p->val.size());
    std::memcpy(p->image.data() + p->off_up, p->up.data(), sizeof(double) * p->up.size());
    *out = p;
    return MRMF_OK;
}

void mrmf_plan_destroy(mrmf_plan plan) { delete plan; }

mrmf_status mrmf_plan_dim(mrmf_plan plan, int64_t* D) {
    if (!plan || !D) return MRMF_E_INVALID_ARG;
    *D = plan->D;
    return MRMF_OK;
}

mrmf_status mrmf_plan_n_offdiag(mrmf_plan plan, int32_t* n) {
    if (!plan || !n) return MRMF_E_INVALID_ARG;
    *n = static_cast<int32_t>(plan->chans.size());
    return MRMF_OK;
}

mrmf_status mrmf_plan_offdiag_terms(mrmf_plan plan, int32_t* out) {
    if (!plan || (!out && !plan->chans.empty())) return MRMF_E_INVALID_ARG;
    for (size_t c = 0; c < plan->chans.size(); ++c) out[c] = plan->chans[c].term;
    return MRMF_OK;
}

mrmf_status mrmf_plan_offsets(mrmf_plan plan, int64_t* out) {
    if (!plan || (!out && !plan->chans.empty())) return MRMF_E_INVALID_ARG;
    for (size_t c = 0; c < plan->chans.size(); ++c) out[c] = plan->chans[c].delta;
    return MRMF_OK;
}

mrmf_status mrmf_plan_workspace_bytes(mrmf_plan plan, size_t* bytes) {
    if (!plan || !bytes) return MRMF_E_INVALID_ARG;
    *bytes = plan->ws_bytes;
    return MRMF_OK;
}

mrmf_status mrmf_plan_upload(mrmf_plan plan, void* d_ws, size_t ws_bytes, mrmf_stream stream) {
    if (!plan || !d_ws || !mrmf::aligned(d_ws, 256)) return MRMF_E_INVALID_ARG;
    if (ws_bytes < plan->ws_bytes) return MRMF_E_WORKSPACE;
    return mrmf::hip_status(hipMemcpyAsync(d_ws, plan->image.data(), plan->ws_bytes,
                                           hipMemcpyHostToDevice, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
