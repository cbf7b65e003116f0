// Decision-tree selector: built-in trees and the JSON loader for trees
// trained by the tuner on timings from this GPU.
#include "selector.hpp"

#include <cctype>
#include <cstdlib>
#include <map>
#include <memory>

#include "../../include/spx.h"

namespace spx {

static const char* kNames[F_COUNT] = {"m",           "n",           "nnz",       "max_row", "min_row",
                                      "avg_row",     "relative_range", "var_nnz_row", "gini",    "nnz_x",
                                      "x_sparsity", "nnz_s",       "m_sparsity", "s_per_x", "counted"};

const char* feature_name(int f) { return (f >= 0 && f < F_COUNT) ? kNames[f] : "?"; }

int feature_id(const std::string& name) {
    for (int i = 0; i < F_COUNT; ++i)
        if (name == kNames[i]) return i;
    return -1;
}

// Builds a tree from (feature, threshold, left, right, class) rows.
static Tree make_tree(std::initializer_list<std::initializer_list<double>> rows) {
    Tree t;
    for (auto& r : rows) {
        auto it = r.begin();
        t.feat.push_back((int32_t)it[0]);
        t.thr.push_back(it[1]);
        t.left.push_back((int32_t)it[2]);
        t.right.push_back((int32_t)it[3]);
        t.cls.push_back((int32_t)it[4]);
    }
    return t;
}

// Trained (tune.py formats-train: the project CART, depth 3, regret-weighted)
// on MI355X timings of the dense-x FP32 SpMV on the 30 tuning matrices:
// best CSR plan, sliced copy, ELL copy and CSR5 copy. Up to 1.17M entries:
// rows of at most 7 entries go to ELL, rows up to 1158 to the sliced copy,
// longer (skewed) rows to CSR5 (R-MAT 2^14 to 2^17 and the small power-law
// matrices, about 10 % under CSR). Beyond: nearly equal rows (relative range
// <= 3.1e-5) to ELL up to 15.7M entries (the 7-point stencils: 128^3 ran
// 25.7 us in ELL against 32.4 in CSR) and to the sliced copy beyond; rows
// whose longest exceeds 17 % of n to CSR5; the rest (the large R-MAT graphs,
// whose CSR kernels read the column-sorted tiles) stay in CSR. On that corpus
// it loses 0.1 % against always taking the fastest format (CSR alone 4.5 %);
// on the FP64 sweep 1.4 % (CSR alone 3.7 %).
Tree format_tree() {
    // rows: feature, threshold, left, right, class (-1 = internal)
    return make_tree({
        {F_NNZ, 1171495.0, 1, 6, -1},
        {F_MAX_ROW, 1158.5, 2, 5, -1},
        {F_MAX_ROW, 7.5, 3, 4, -1},
        {0, 0, 0, 0, 2},
        {0, 0, 0, 0, 1},
        {0, 0, 0, 0, 3},
        {F_REL_RANGE, 3.07220458984375e-05, 7, 10, -1},
        {F_NNZ, 15679488.0, 8, 9, -1},
        {0, 0, 0, 0, 2},
        {0, 0, 0, 0, 1},
        {F_REL_RANGE, 0.17117210571289063, 11, 12, -1},
        {0, 0, 0, 0, 0},
        {0, 0, 0, 0, 3},
    });
}

// Untrained defaults, written on host-known features only so that run()
// needs no device-to-host sync: vector density picks the pattern
// (column-major when sparse, row-major with validation in between, SpMV
// when dense); an unequal row-length distribution (Gini) picks the
// balanced distribution; few vector entries pick atomics, a y that fits in
// LDS the privatized atomics, otherwise the bucket write-back.
Selector builtin_selector() {
    Selector s;
    s.pattern = make_tree({
        {F_X_SPARSITY, 0.1, 1, 2, -1},
        {0, 0, 0, 0, SPX_PAT_CSC_SPMSPV},
        {F_X_SPARSITY, 0.3, 3, 4, -1},
        {0, 0, 0, 0, SPX_PAT_CSR_SPMSPV},
        {0, 0, 0, 0, SPX_PAT_SPMV},
    });
    for (int p = 0; p < 3; ++p)
        s.distribution[p] = make_tree({
            {F_GINI, 0.5, 1, 2, -1},
            {0, 0, 0, 0, SPX_DIST_DIRECT},
            {0, 0, 0, 0, SPX_DIST_BALANCED},
        });
    s.writeback = make_tree({
        {F_NNZ_X, 2048, 1, 2, -1},
        {0, 0, 0, 0, SPX_WB_ATOMIC},
        {F_M, 16384, 3, 4, -1},
        {0, 0, 0, 0, SPX_WB_LDS_ATOMIC},
        {0, 0, 0, 0, SPX_WB_BUCKET},
    });
    s.source = "builtin";
    return s;
}

// ------------------------------------------------------------- tiny JSON
namespace {

struct JVal {
    enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<std::shared_ptr<JVal>> arr;
    std::map<std::string, std::shared_ptr<JVal>> obj;
    const JVal* get(const std::string& k) const {
        auto it = obj.find(k);
        return it == obj.end() ? nullptr : it->second.get();
    }
};

struct Parser {
    const std::string& s;
    size_t i = 0;
    std::string err;
    explicit Parser(const std::string& t) : s(t) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool expect(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        err = std::string("expected '") + c + "' at offset " + std::to_string(i);
        return false;
    }
    std::shared_ptr<JVal> value() {
        ws();
        if (i >= s.size()) {
            err = "unexpected end";
            return nullptr;
        }
        auto v = std::make_shared<JVal>();
        char c = s[i];
        if (c == '{') {
            ++i;
            v->kind = JVal::OBJ;
            ws();
            if (i < s.size() && s[i] == '}') {
                ++i;
                return v;
            }
            while (true) {
                ws();
                auto k = value();
                if (!k || k->kind != JVal::STR) {
                    if (err.empty()) err = "object key must be a string";
                    return nullptr;
                }
                if (!expect(':')) return nullptr;
                auto x = value();
                if (!x) return nullptr;
                v->obj[k->str] = x;
                ws();
                if (i < s.size() && s[i] == ',') {
                    ++i;
                    continue;
                }
                if (!expect('}')) return nullptr;
                return v;
            }
        }
        if (c == '[') {
            ++i;
            v->kind = JVal::ARR;
            ws();
            if (i < s.size() && s[i] == ']') {
                ++i;
                return v;
            }
            while (true) {
                auto x = value();
                if (!x) return nullptr;
                v->arr.push_back(x);
                ws();
                if (i < s.size() && s[i] == ',') {
                    ++i;
                    continue;
                }
                if (!expect(']')) return nullptr;
                return v;
            }
        }
        if (c == '"') {
            ++i;
            v->kind = JVal::STR;
            while (i < s.size() && s[i] != '"') {
                if (s[i] == '\\' && i + 1 < s.size()) ++i;
                v->str.push_back(s[i++]);
            }
            if (i >= s.size()) {
                err = "unterminated string";
                return nullptr;
            }
            ++i;
            return v;
        }
        if (s.compare(i, 4, "true") == 0) {
            i += 4;
            v->kind = JVal::BOOL;
            v->b = true;
            return v;
        }
        if (s.compare(i, 5, "false") == 0) {
            i += 5;
            v->kind = JVal::BOOL;
            return v;
        }
        if (s.compare(i, 4, "null") == 0) {
            i += 4;
            return v;
        }
        const char* start = s.c_str() + i;
        char* end = nullptr;
        v->num = std::strtod(start, &end);
        if (end == start) {
            err = "bad value at offset " + std::to_string(i);
            return nullptr;
        }
        v->kind = JVal::NUM;
        i += (size_t)(end - start);
        return v;
    }
};

bool tree_from_json(const JVal* t, Tree* out, int n_classes_max, std::string* err) {
    if (!t || t->kind != JVal::OBJ) {
        *err = "tree must be an object";
        return false;
    }
    const JVal* nodes = t->get("nodes");
    if (!nodes || nodes->kind != JVal::ARR || nodes->arr.empty()) {
        *err = "tree needs a non-empty 'nodes' array";
        return false;
    }
    Tree tr;
    const int n = (int)nodes->arr.size();
    for (auto& row : nodes->arr) {
        if (row->kind != JVal::ARR || row->arr.size() != 5) {
            *err = "node must be [feature, threshold, left, right, class]";
            return false;
        }
        int f;
        if (row->arr[0]->kind == JVal::STR)
            f = feature_id(row->arr[0]->str);
        else
            f = (int)row->arr[0]->num;
        const int l = (int)row->arr[2]->num, r = (int)row->arr[3]->num, c = (int)row->arr[4]->num;
        if (c < 0) {
            if (f < 0 || f >= F_COUNT || l <= 0 || r <= 0 || l >= n || r >= n) {
                *err = "internal node with a bad feature or child index";
                return false;
            }
        } else if (c >= n_classes_max) {
            *err = "leaf class out of range";
            return false;
        }
        tr.feat.push_back(f < 0 ? 0 : f);
        tr.thr.push_back(row->arr[1]->num);
        tr.left.push_back(l);
        tr.right.push_back(r);
        tr.cls.push_back(c);
    }
    *out = tr;
    return true;
}

}  // namespace

bool parse_selector_json(const std::string& text, Selector* out, std::string* err) {
    Parser p(text);
    auto root = p.value();
    if (!root) {
        *err = "json: " + p.err;
        return false;
    }
    if (root->kind != JVal::OBJ) {
        *err = "json: top level must be an object";
        return false;
    }
    Selector s = builtin_selector();
    if (!tree_from_json(root->get("pattern"), &s.pattern, 3, err)) return false;
    const JVal* d = root->get("distribution");
    if (!d || d->kind != JVal::OBJ) {
        *err = "json: 'distribution' must map pattern names to trees";
        return false;
    }
    const char* pn[3] = {"spmv", "csr_spmspv", "csc_spmspv"};
    for (int i = 0; i < 3; ++i)
        if (!tree_from_json(d->get(pn[i]), &s.distribution[i], 2, err)) return false;
    if (!tree_from_json(root->get("writeback"), &s.writeback, 6, err)) return false;
    const JVal* lz = root->get("lazy");
    s.lazy = lz && lz->kind == JVal::BOOL && lz->b;
    const JVal* src = root->get("source");
    s.source = (src && src->kind == JVal::STR) ? src->str : "json";
    *out = s;
    return true;
}

}  // namespace spx
