// Constraint bytecode shared by the compiler (host) and the interpreter (device).
//
// One 32-bit word per instruction: opcode in bits 0..7, a signed 24-bit
// immediate in bits 8..31.  OP_CONST64 is followed by two words (low, high).
// Each constraint is one stack program that leaves one value; the
// configuration satisfies it iff that value is non-zero and no step raised.
#pragma once

#define CT_MAX_PROGRAMS 64

enum ct_opcode {
    OP_PARAM = 1,    // push value of parameter imm
    OP_CONST = 2,    // push imm
    OP_CONST64 = 3,  // push the next two words as int64
    OP_NEG = 4, OP_ABS = 5, OP_NOT = 6,
    OP_ADD = 7, OP_SUB = 8, OP_MUL = 9, OP_FDIV = 10, OP_MOD = 11,
    OP_MIN = 12, OP_MAX = 13,
    OP_LT = 14, OP_LE = 15, OP_GT = 16, OP_GE = 17, OP_EQ = 18, OP_NE = 19,
    OP_AND = 20, OP_OR = 21,
    OP_LAST = 21
};
