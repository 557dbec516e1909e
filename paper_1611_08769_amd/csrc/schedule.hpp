// Lowering of a gate netlist to device work: which gate outputs become
// ciphertexts in memory, which ciphertext-ciphertext products run at which
// level, and which memory slot each intermediate ciphertext occupies.
//
// Every gate of the circuit is one of (paper, section "Notation and
// Background": addition and multiplication of ciphertexts, NAND) the forms
//   AND = P,  XOR = L + R - 2P,  OR = L + R - P,  NOT = G - X,  XADD = X + Y
// with P = BitDecomp(L) R mod q the product of its two operands.  A product
// is computed once per ordered operand pair; every ciphertext derived from it
// by a linear form a L + b R + c P + g G + e E (E another ciphertext already
// in memory) is written by the product's epilogue.  Linear forms with no
// product (NOT of an input, copies of outputs) run as separate linear items.
#pragma once
#include <cstdint>
#include <vector>

#include "netlist.hpp"

namespace sfft {

constexpr int kMaxOut = 4;   // epilogue outputs per product item
constexpr int kMaxE = 2;     // distinct extra operands per product item
constexpr int kMaxCoef = 3;  // bound on |a|, |b|, |c|, |g|, |e| of every output form

// Ciphertext reference: buffer in bits 31..29, index in bits 28..0.
enum CtBuf : uint32_t { B_IN = 0, B_OUT = 1, B_WS = 2, B_AUX = 3 };
inline int32_t ct_ref(uint32_t buf, uint32_t idx) { return (int32_t)((buf << 29) | idx); }

struct ProdItem {
    int32_t L, R;          // operand refs
    int32_t nout;
    int32_t dst[kMaxOut];  // output refs
    int32_t E[kMaxOut];    // extra operand refs (or -1)
    int8_t cL[kMaxOut], cR[kMaxOut], cP[kMaxOut], cG[kMaxOut], cE[kMaxOut];
    int32_t pad;
};

struct LinItem {
    int32_t dst;
    int32_t X, Y;          // refs or -1
    int8_t cX, cY, cG, pad;
};

struct LevelWork {
    int64_t prod_begin = 0, prod_count = 0;   // into Schedule::prods
    // linear passes after the products of this level, one per sub-level
    std::vector<std::pair<int64_t, int64_t>> lin;  // (begin, count) into Schedule::lins
};

struct Schedule {
    std::vector<ProdItem> prods;
    std::vector<LinItem> lins;
    std::vector<LevelWork> levels;   // levels[0] has only linear passes (before any product)
    std::vector<LinItem> final_lins; // outputs that are constants, inputs or repeated
    int64_t n_slots = 0;             // workspace ciphertexts
    int64_t n_products = 0;
    int64_t max_level_products = 0;
};

// Bounds on the live set of a schedule (0: none).  max_slots bounds the
// workspace ciphertexts live at once, max_level_products the product items
// of one level (each level's right operands take transposition scratch),
// max_window how far (in order of first appearance) a product may run ahead
// of the first one not yet run, which keeps the schedule from opening more
// independent parts of the circuit (rows of an image) than fit.
struct LiveLimit {
    int64_t max_slots = 0;
    int64_t max_level_products = 0;
    int64_t max_window = 0;
};

// Build the schedule for a (DCE'd, optionally shared) netlist: levels as
// soon as possible, or, under a limit, by list scheduling within it.
Schedule lower(const Compact& c, const LiveLimit& lim = LiveLimit{});

}  // namespace sfft
