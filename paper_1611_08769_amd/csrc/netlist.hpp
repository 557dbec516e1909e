// Gate netlist of the encrypted fixed-point FFT: construction, dead-code
// elimination, structural sharing, canonical hash and the worst-case noise
// bound that sizes the modulus.
//
// Paper, section "FFT in FHE": bits are encrypted individually; the NOT, AND,
// OR and XOR gates (Lemma "binary gates") form half and full adders
// (Lemmas "half adder", "full adder"), ripple-carry addition and subtraction
// by inverting the subtrahend with carry-in 1 (Lemma "add/subtract"), a
// Wallace-tree multiplier on sign-extended operands whose middle bits give the
// fixed-point product (Lemmas "integer multiplication", "fixed
// multiplication"), and the radix-2 butterflies of a decimation-in-time FFT
// with plaintext twiddles and plaintext bit reversal (Lemma "evaluation").
#pragma once
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace sfft {

enum NodeType : int8_t {
    T_IN = 0, T_C0 = 1, T_C1 = 2, T_NOT = 3, T_AND = 4, T_XOR = 5, T_OR = 6, T_XADD = 7, T_NAND = 8
};
// node types evaluated through the product of their two operands
inline bool is_product_type(int8_t t) { return t == T_AND || t == T_XOR || t == T_OR || t == T_NAND; }

constexpr int32_t kZero = 0, kOne = 1;
enum AdderMode { kRipple = 0, kCsa = 1 };

struct Shape {
    int dims;  // 1 or 2
    int len;   // points (1D) or image side (2D); power of two
    int F;     // word width
    int f;     // fractional bits
    bool is_complex;
    bool nand_only = false;  // every gate a NAND (the paper's literal circuit)
    int points() const { return dims == 1 ? len : len * len; }
    int n_inputs() const { return points() * (is_complex ? 2 : 1) * F; }
    int n_outputs() const { return points() * 2 * F; }
};

// Plaintext twiddle exp(-2 pi i j / m) in Q(., f), rounded half away from zero.
void twiddle(int j, int m, int f, int64_t* cr, int64_t* ci);

class Netlist {
public:
    std::vector<int8_t> t;
    std::vector<int32_t> a, b;
    std::vector<int32_t> outputs;
    int32_t n_inputs = 0;

    // nand_only: NOT x = NAND(x, x), AND = NOT NAND, OR(l, r) = NAND(NOT l,
    // NOT r), XOR(l, r) = NAND(NAND(l, t), NAND(r, t)) with t = NAND(l, r),
    // and a full adder's carry is the OR of its two half-adder carries
    // (paper, Lemmas "binary gates" and "full adder")
    explicit Netlist(bool nand_only = false);
    bool nand_only;
    int32_t input();
    int32_t NAND(int32_t l, int32_t r);
    int32_t NOT(int32_t x);
    int32_t AND(int32_t l, int32_t r);
    int32_t XOR(int32_t l, int32_t r);
    int32_t OR(int32_t l, int32_t r);
    int32_t XADD(int32_t x, int32_t y);
    std::pair<int32_t, int32_t> HA(int32_t x, int32_t y);           // (sum, carry)
    std::pair<int32_t, int32_t> FA(int32_t x, int32_t y, int32_t c, AdderMode mode);
    std::vector<int32_t> add(const std::vector<int32_t>& x, const std::vector<int32_t>& y);
    std::vector<int32_t> sub(const std::vector<int32_t>& x, const std::vector<int32_t>& y);
    std::vector<int32_t> mul_const(const std::vector<int32_t>& x, int64_t c, int f);

    struct Cplx { std::vector<int32_t> re, im; };
    std::vector<Cplx> fft1d(const std::vector<Cplx>& xs, int f);

private:
    int32_t node(int8_t type, int32_t x, int32_t y);
};

Netlist build_fft_netlist(const Shape& s);

// Nodes reachable from the outputs (inputs always kept), renumbered densely
// in construction order.  Constants keep ids 0 and 1.
struct Compact {
    std::vector<int8_t> t;
    std::vector<int32_t> a, b;
    std::vector<int32_t> outputs;
    int32_t n_inputs = 0;
    size_t size() const { return t.size(); }
};

Compact compact(const Netlist& nl);

// Merge nodes with identical type and identical (already merged) operands.
// Gate evaluation is deterministic, so every merged node carries the same
// ciphertext as each of the nodes it replaces.
Compact share(const Compact& c);

// SHA-256 (FIPS 180-4) of the node list: per node (u8 type, i32 a, i32 b)
// little-endian, then u32 output count and i32 output ids.
std::string netlist_hash(const Compact& c);

struct NetStats {
    int64_t nodes, products, gates, nots, depth, max_width;
};
NetStats netlist_stats(const Compact& c);

// Least k (multiple of 32) whose noise rule holds: bitlen(Bmax) + 3 <= k with
// Nct = (n_lwe + 1) k.  Returns -1 if none below k_limit.
int choose_k(const Compact& c, int n_lwe, int k_limit = 8192);
// bitlen(Bmax) + 3 at a given Nct.
int noise_bits(const Compact& c, int64_t nct);

}  // namespace sfft
