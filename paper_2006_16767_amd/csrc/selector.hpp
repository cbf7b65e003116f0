// Decision-tree kernel selector (Section 5 and Section 6.2-6.3).
//
// Three models are evaluated as a cascade: the computing-pattern tree, then
// the workload-distribution tree of the chosen pattern, then (column-major
// pattern only) the write-back tree. Features (Table 1) are produced lazily
// through a callback, so a tree that decides on m, n, nnz or nnz_x never
// triggers the device reduction behind nnz_s.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace spx {

// Feature ids, in the order of Table 1.
enum Feature {
    F_M = 0,
    F_N,
    F_NNZ,
    F_MAX_ROW,
    F_MIN_ROW,
    F_AVG_ROW,
    F_REL_RANGE,
    F_VAR_ROW,
    F_GINI,
    F_NNZ_X,
    F_X_SPARSITY,
    F_NNZ_S,
    F_M_SPARSITY,
    F_S_PER_X,  // nnz_s / max(1, nnz_x): mean length of the selected columns (derived, not in Table 1)
    F_COUNTED,  // 1 when the vector's counts (nnz_s) are already known, else 0: lets a later tree of the
                // cascade use them for free once an earlier one paid for them (not in Table 1)
    F_COUNT
};

const char* feature_name(int f);
int feature_id(const std::string& name);

// A binary tree in flat arrays; node i is a leaf when cls[i] >= 0.
// Internal nodes: go left when feature value <= thr.
struct Tree {
    std::vector<int32_t> feat, left, right, cls;
    std::vector<double> thr;
    bool empty() const { return cls.empty(); }
    template <typename FeatFn>
    int eval(FeatFn&& f) const {
        int i = 0;
        for (int guard = 0; guard < 64; ++guard) {
            if (cls[i] >= 0) return cls[i];
            i = f(feat[i]) <= thr[i] ? left[i] : right[i];
        }
        return cls[i] >= 0 ? cls[i] : 0;
    }
};

struct Selector {
    Tree pattern;          // classes: spx_pattern
    Tree distribution[3];  // per pattern; classes: spx_distribution
    Tree writeback;        // classes: spx_writeback
    std::string source = "builtin";
    // lazy trees decide run() and select_kernel(): they may test nnz_s (or
    // m_sparsity, s_per_x), computed on the device only when the walk reaches
    // such a node (the tuner charges that round trip in training)
    bool lazy = false;
    // true when an internal node of any tree tests nnz_s, m_sparsity or
    // s_per_x, the features that need the vector's column lengths
    bool reads_nnz_s() const {
        const Tree* ts[5] = {&pattern, &distribution[0], &distribution[1], &distribution[2], &writeback};
        for (const Tree* t : ts)
            for (size_t i = 0; i < t->cls.size(); ++i)
                if (t->cls[i] < 0 &&
                    (t->feat[i] == F_NNZ_S || t->feat[i] == F_M_SPARSITY || t->feat[i] == F_S_PER_X))
                    return true;
        return false;
    }
};

Selector builtin_selector();

// Storage-format pre-selector: class 0 keeps CSR only, class 1 adds the
// sliced ELLPACK copy, class 2 the ELLPACK copy, class 3 the CSR5 copy, for
// the format expected to run the SpMV fastest. Feature ids 0-8 are the Table 1 matrix features
// (F_M .. F_GINI), kFmtPadding the padding ratio of the sliced copy
// (cells / nnz; ratio() computes it on first use, from a host copy of
// row_ptr), kFmtEllPadding that of the ELL copy (max_row * m / nnz, from the
// features).
constexpr int kFmtPadding = 9;
constexpr int kFmtEllPadding = 10;
Tree format_tree();
template <typename RatioFn>
int format_choice(const double* feat, RatioFn&& ratio) {
    static const Tree t = format_tree();
    const double ell = feat[F_NNZ] > 0 ? feat[F_MAX_ROW] * feat[F_M] / feat[F_NNZ] : 1.0;
    const int c = t.eval([&](int f) { return f < kFmtPadding ? feat[f] : f == kFmtPadding ? ratio() : ell; });
    return c >= 0 && c <= 3 ? c : 0;
}
// Parses the tuner's JSON. Returns false with a message on error.
bool parse_selector_json(const std::string& text, Selector* out, std::string* err);

}  // namespace spx
