// Internal definitions shared by the host runtime and the HIP kernels.
#pragma once

#include <stdint.h>

namespace gpx {

// ---------------------------------------------------------------------------
// Lowered tree code.  A tree becomes a list of stack-operand instructions
// (the paper's linear form, section 5): each function reads its operands
// from a case input X, a constant C or the stack S and pushes its result.
// Two 32-bit words per instruction:
//   w0 bits 0-3   op    (GP function 0-9 or 12-14, OP_IF, or OP_PUSH)
//      bits 4-7   mode  (where the operands come from, see below)
//      bits 8-15  feature index of operand A (X modes)
//      bits 16-23 feature index of operand B (X modes)
//      bits 24-31 stack height after the instruction (a check value)
//   w1            constant operand, binary32 bits (C modes)
// h is the stack height before the instruction; s[0] is the bottom.
// ---------------------------------------------------------------------------
enum : uint32_t { OP_PUSH = 15 };
// The three-operand IF (public opcode GP_IF) in the 4-bit op field: 10 is
// NAND, a function of the Boolean set only, so no arithmetic tree uses it.
enum : uint32_t { OP_IF = 10 };

enum : uint32_t {
    M_SS = 0,   // A = s[h-2], B = s[h-1]  -> s[h-2], h-1
    M_SSR = 1,  // A = s[h-1], B = s[h-2]  -> s[h-2], h-1   (right subtree ran first)
    M_SX = 2,   // A = s[h-1], B = X_b     -> s[h-1]
    M_XS = 3,   // A = X_a,    B = s[h-1]  -> s[h-1]
    M_SC = 4,   // A = s[h-1], B = c       -> s[h-1]
    M_CS = 5,   // A = c,      B = s[h-1]  -> s[h-1]
    M_XX = 6,   // push op(X_a, X_b)
    M_XC = 7,   // push op(X_a, c)
    M_CX = 8,   // push op(c, X_b)
    M_S = 9,    // unary, in place on s[h-1]
    M_X = 10,   // unary on X_a, pushed (OP_PUSH: push X_a)
    M_C = 11,   // unary on c, pushed   (OP_PUSH: push c)
    M_S3 = 12,  // three operands s[h-3], s[h-2], s[h-1] -> s[h-3], h-2; operand A is the value at
                //   position fa (0 = s[h-3]), B at position fb, C at the remaining one (IF only)
};

inline uint32_t enc_w0(uint32_t op, uint32_t mode, uint32_t fa, uint32_t fb, uint32_t h_after) {
    return (op & 15u) | ((mode & 15u) << 4) | ((fa & 255u) << 8) | ((fb & 255u) << 16) |
           ((h_after & 255u) << 24);
}

// ---------------------------------------------------------------------------
// Per-program record on the device (32 bytes).
// ---------------------------------------------------------------------------
enum : uint32_t { FORM_TREE = 0, FORM_LINEAR = 1 };

struct DevProg {
    uint32_t code_off;     // first word of the program in the code array
    uint32_t len;          // instructions (trees: 2 words each; linear: 1 word each,
                           //   followed by the program's constants)
    uint32_t meta;         // bit 0 form; bits 8-15 stack depth (tree) or n_reg (linear)
    uint32_t reserved0;
    uint64_t reserved1;
    uint64_t row;          // program index within its population (per-case output row)
};
static_assert(sizeof(DevProg) == 32, "DevProg layout");

// ---------------------------------------------------------------------------
// Host lowering (lower.cpp)
// ---------------------------------------------------------------------------
struct TreeLowering {
    int32_t n_nodes = 0;
    int32_t n_instr = 0;
    int32_t max_depth = 0;
    int32_t stack_fetches = 0;
    int32_t n_values = 0;
    int32_t n_reversed = 0;
};

// Function sets a tree may use: the arithmetic set {+,-,*,/p,sin,cos,exp,log}
// with variables and constants, or the Boolean set {AND,OR,NAND,NOR} with
// variables only.
enum : int { OPSET_REAL = 0, OPSET_BOOL = 1 };

// Validates one prefix tree and appends its lowered words to `out` (may be
// null to only compute the statistics).  Returns 0 or a gp_status code and
// writes a message into `err` (at least 256 bytes).  cst may be null for
// the Boolean set.
int lower_tree(const int32_t* tok, const float* cst, int64_t n, int32_t n_feat,
               uint32_t* out, TreeLowering* st, char* err, int opset = OPSET_REAL);

// Validates one register linear program.
int check_linear(const uint32_t* code, int64_t n, int64_t n_cst, int32_t n_reg, int32_t n_feat,
                 char* err);

}  // namespace gpx
