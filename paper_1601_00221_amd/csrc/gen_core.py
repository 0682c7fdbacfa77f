"""Generate the hand-written gfx950 interpreter core (a build step).

    python gen_core.py OUT_DIR

Writes ``core_gen.inc``: for every kernel variant (T case slots per lane, D
stack levels, NF feature slots) one inline-asm interpreter loop plus the
host-side table naming its handlers.

Design.  The whole two-dimensional stack (level l, slot j), the registers of
a linear program and the wave's case tile live in a VGPR range the compiler
does not allocate (the kernel caps the compiler's own VGPRs).  Offsets in
that range, relative to its first register V0:

    stack level l / linear register r, slot j :  l*T + j        (l < RB)
    feature f, slot j                          :  RB*T + f*T + j  (f < NF)

with RB = max(8, D) register/stack levels (RB = D in the Boolean kernels,
which run trees only).

A program is a list of 16-byte instructions

    dword 0-1  absolute address of the handler that executes it
    dword 2    operand offsets (byte 0 = first index, byte 1 = second index;
               for an exit: A, B, destination offsets and the operation)
    dword 3    constant operand (binary32 bits)

A handler loads the next instruction with one scalar load, executes its own
T vector instructions with the wave-uniform operand offset applied through
the gfx9 VGPR index mode (one index per instruction; the other operands of
the handler are fixed registers, so handlers are specialised on stack level
or register number), waits for the load and jumps to the next handler's
address.  Every lane runs the same program, so the jump is uniform.
Protected division and the classification functions have handlers of
their own that read their operands at any offsets.  Work the core does not
do itself (sin/cos/exp/log, the end of a program) leaves the asm block
through the exit handler with the instruction's payload; the compiled
kernel does it and re-enters.

Fixed SGPRs used by the block: s[60:61] code base, s62 byte offset of the
current instruction, s63 probe flag, s[64:71] the current and next
instruction records, s72-s74 and s79 a constant copy and index temporaries,
s[80:81] the division threshold or a compare's mask, vcc flags, s75 the
end of the program's code and s78 the loads in flight for its burst load
into the scalar cache, s[76:77] table address (probe).
"""
import os
import sys

SLOT = 64                 # bytes per handler slot; longer handlers take several
LIN_REGS = 8              # register slots reserved for linear programs (and stack levels)

# (T, D, NF, NCV, MODE) variants: T case slots per lane, D stack levels, NF
# feature slots, NCV VGPRs left to the compiler (the core owns v[NCV ...]),
# MODE = 0 for the arithmetic function set with the sin/cos/exp/log code,
# 1 without that code (for programs that use none; its compiled part is
# small, so nothing spills), 2 for the Boolean function set (slots are
# 32-bit words of bit-packed cases), 3 like 1 for trees only (no linear
# handlers or registers: a handler table half the size, and the stack
# levels start the VGPR range), 4 like 0 for trees only (the core of mode
# 3 with the sin/cos/exp/log code: room for many feature slots).  Work that
# leaves the core (sin/cos/exp/log in binary64) runs in the compiler's VGPRs:
# programs rich in it take a variant with room for it.
VARIANTS = [
    (8, 6, 8, 40, 0),
    (8, 6, 8, 128, 0),
    (8, 8, 8, 40, 0),
    (4, 8, 8, 40, 0),
    (4, 8, 16, 40, 0),
    (4, 12, 32, 40, 0),
    (8, 8, 8, 128, 0),
    (4, 8, 16, 128, 0),
    (4, 12, 32, 80, 0),
    (4, 8, 8, 64, 0),
    (4, 8, 8, 96, 0),
    (4, 8, 16, 64, 0),
    (8, 6, 8, 40, 1),
    (8, 8, 8, 40, 1),
    (4, 8, 16, 40, 1),
    (4, 12, 32, 40, 1),
    (8, 6, 8, 56, 3),
    (8, 8, 8, 40, 3),
    (4, 8, 16, 48, 3),
    (4, 8, 44, 48, 4),
    (8, 6, 20, 48, 2),
    (8, 8, 20, 32, 2),
    (4, 12, 32, 40, 2),
    # deep programs: every tree of at most GP_MAX_LEN nodes needs at most 20
    # levels (15 without IF), 16 for the binary Boolean set; with more than 32
    # features the deepest that fits beside them is 12
    (4, 20, 32, 40, 0),
    (4, 12, 44, 32, 4),
    (4, 16, 32, 40, 2),
    # Boolean, 4 waves per SIMD: 5 % faster than (8, 6, 20, 48) on the 20-multiplexer (2 waves, the same 16
    # slots per SIMD); 3-wave forms of it were slower
    (4, 6, 20, 24, 2),
    # 4 waves per SIMD at T = 4 for the functions that stay in the core: the Shuttle shape's 9 inputs (16 %
    # faster than (4, 8, 16, 48) with 3 waves) and register programs over 16 features (13 % faster than
    # (4, 8, 16, 40))
    (4, 8, 12, 48, 3),
    (4, 8, 16, 32, 1),
]


def vname(v):
    """Kernel name suffix of a variant: T_D_NF_NCV, plus _a when it has no
    sin/cos/exp/log code, _at when it also runs trees only, _t for trees only
    with that code, and _b for the Boolean function set."""
    return "%d_%d_%d_%d%s" % (v[0], v[1], v[2], v[3], ("", "_a", "_b", "_at", "_t")[v[4]])

OPS = {"add": "v_add_f32_e32", "sub": "v_sub_f32_e32", "mul": "v_mul_f32_e32"}
OP_ID = {"add": 0, "sub": 1, "mul": 2}
# Boolean functions (ids as the tree opcodes GP_AND .. GP_NOR).  AND and OR
# are one VOP2 operation; NAND and NOR one v_bitop3_b32, whose truth table
# has bit (4 s0 + 2 s1 + s2) set where the result is 1 (the third source is
# ignored by these tables).
BOOL_OPS = {"and": "v_and_b32_e32", "or": "v_or_b32_e32", "nand": 0x3F, "nor": 0x03}
BOOL_ID = {"and": 8, "or": 9, "nand": 10, "nor": 11}


def bool_op(op, d, a, b):
    """d = a op b; a and b keep their positions as first and second source."""
    ins = BOOL_OPS[op]
    if isinstance(ins, str):
        return "%s %s, %s, %s" % (ins, d, a, b)
    return "v_bitop3_b32 %s, %s, %s, %s bitop3:0x%x" % (d, a, b, b, ins)


def reg_levels(D, mode):
    """Register/stack levels before the features: linear programs need
    LIN_REGS registers; Boolean and trees-only kernels have none."""
    return D if mode >= 2 else max(LIN_REGS, D)

# handler kinds (keep in sync with the generated enum below)
KINDS = ["EXIT", "SS", "SSR", "SX", "XS", "SC", "CS", "XX", "XX2", "XC", "CX", "PUSHX", "PUSHC",
         "RR", "XR", "FF", "CR", "RC", "MOVC", "MOVX", "DVV", "DVC", "DCV", "CVV", "CVC", "CCV", "IF3"]
# Protected division runs in the core: a / b with a and b at any two offsets
# (DVV), b the constant (DVC) or a the constant (DCV), the result to a third
# offset.  Its temporaries are the last DIV_TMP registers of the compiler's
# range (clobbered by the block), its flags vcc, its indexes s73/s74/s79 and
# the protection threshold s80.
DIV_TMP = 7
DIV_THRESHOLD = 0x358637BD       # 1e-6f: |b| below it gives 1
K = {k: i for i, k in enumerate(KINDS)}


def vr(n):
    assert 0 <= n < 256, n
    return "v%d" % n


VOP3_ONLY = ("v_bitop3", "v_div_scale_f32", "v_fma_f32", "v_div_fmas_f32", "v_div_fixup_f32")


def insn_bytes(text):
    """Encoded size of an instruction the handlers use: scalar loads, VOP3
    encodings and a scalar move of a literal take 8 bytes, everything else 4."""
    if text.startswith(("s_load",) + VOP3_ONLY) or text.split(" ")[0].endswith("_e64"):
        return 8
    if text.startswith("s_mov_b32") and "0x" in text:
        return 8
    return 4


class Handler:
    def __init__(self, kind, op=0, p1=0, p2=0):
        self.kind, self.op, self.p1, self.p2 = kind, op, p1, p2
        self.lines = []
        self.size = 0
        self.phases = None      # (phase A lines, phase B lines) of a handler written per phase

    def emit(self, text, nbytes):
        self.lines.append(text)
        self.size += nbytes


def gen_variant(T, D, NF, NCV, mode=0):
    V0 = NCV
    FO = reg_levels(D, mode) * T       # register/stack block, then the features
    assert FO + NF * T <= 256, "index range exceeds 8 bits"
    assert V0 + FO + NF * T <= 256
    assert NCV % 8 == 0
    tag = "T%dD%dF%dV%d%s" % (T, D, NF, NCV, {2: "B", 3: "R", 4: "R"}.get(mode, ""))
    hs = []

    def prologue(h, const=False, second_index=False, index=None):
        """Save what the handler still needs from the current record (the
        next record's load overwrites s[64:67]), then start that load.  A
        handler with one index turns the index mode on straight from the
        payload, before the load is issued."""
        if const:
            h.emit("s_mov_b32 s72, s67", 4)
        if index == "off":
            h.emit("s_set_gpr_idx_off", 4)
        elif index is not None:
            idx_on(h, "s66", index)
        else:
            h.emit("s_mov_b32 s70, s66", 4)
        if second_index:
            h.emit("s_lshr_b32 s71, s66, 8", 4)
        h.emit("s_add_u32 s62, s62, 16", 4)
        h.emit("s_load_dwordx4 s[64:67], s[60:61], s62", 8)

    def idx_on(h, sreg, modes):
        h.emit("s_set_gpr_idx_on %s, gpr_idx(%s)" % (sreg, ",".join(modes)), 4)

    def epilogue(h):
        h.emit("s_waitcnt lgkmcnt(0)", 4)
        h.emit("s_setpc_b64 s[64:65]", 4)

    def valu(h, text):
        h.emit(text, insn_bytes(text))

    # ---------------------------------------------------------------- exit
    h = Handler(K["EXIT"])
    h.emit("s_set_gpr_idx_off", 4)
    h.emit("s_branch .Lgpx_end_%s" % tag, 4)
    hs.append(h)

    if mode == 2:
        bool_handlers(hs, T, D, V0, FO, prologue, idx_on, epilogue, valu)
        return finish(hs, tag, V0, FO)

    # ---------------------------------------------------------------- trees
    for op in ("add", "sub", "mul"):
        h = Handler(K["SS"], OP_ID[op])            # s[h-2] = s[h-2] op s[h-1]; index (h-2)*T
        prologue(h, index=["SRC0", "SRC1", "DST"])
        for j in range(T):
            valu(h, "%s %s, %s, %s" % (OPS[op], vr(V0 + j), vr(V0 + j), vr(V0 + T + j)))
        epilogue(h)
        hs.append(h)
    h = Handler(K["SSR"], OP_ID["sub"])            # s[h-2] = s[h-1] - s[h-2]
    prologue(h, index=["SRC0", "SRC1", "DST"])
    for j in range(T):
        valu(h, "v_sub_f32_e32 %s, %s, %s" % (vr(V0 + j), vr(V0 + T + j), vr(V0 + j)))
    epilogue(h)
    hs.append(h)
    for op in ("add", "sub", "mul"):
        for l in range(D):
            h = Handler(K["SX"], OP_ID[op], l)     # s[l] = s[l] op x[b]; index = feature offset
            prologue(h, index=["SRC1"])
            for j in range(T):
                r = vr(V0 + l * T + j)
                valu(h, "%s %s, %s, %s" % (OPS[op], r, r, vr(V0 + j)))
            epilogue(h)
            hs.append(h)
    for l in range(D):
        h = Handler(K["XS"], OP_ID["sub"], l)      # s[l] = x[a] - s[l]
        prologue(h, index=["SRC0"])
        for j in range(T):
            r = vr(V0 + l * T + j)
            valu(h, "v_sub_f32_e32 %s, %s, %s" % (r, vr(V0 + j), r))
        epilogue(h)
        hs.append(h)
    for op, ins in (("add", "v_add_f32_e32"), ("mul", "v_mul_f32_e32"), ("sub", "v_subrev_f32_e32")):
        h = Handler(K["SC"], OP_ID[op])            # s[l] = s[l] op c; index l*T
        prologue(h, const=True, index=["SRC1", "DST"])
        for j in range(T):
            valu(h, "%s %s, s72, %s" % (ins, vr(V0 + j), vr(V0 + j)))
        epilogue(h)
        hs.append(h)
    h = Handler(K["CS"], OP_ID["sub"])             # s[l] = c - s[l]
    prologue(h, const=True, index=["SRC1", "DST"])
    for j in range(T):
        valu(h, "v_sub_f32_e32 %s, s72, %s" % (vr(V0 + j), vr(V0 + j)))
    epilogue(h)
    hs.append(h)
    if NF <= 8:
        # push x[a] op x[b] at level l: both sources relative to one index a*T,
        # the second one displaced by delta = b - a feature rows
        for op in ("add", "mul", "sub"):
            deltas = range(0, NF) if op != "sub" else range(-(NF - 1), NF)
            for l in range(D):
                for dl in deltas:
                    h = Handler(K["XX"], OP_ID[op], l, dl)
                    prologue(h, index=["SRC0", "SRC1"])
                    for j in range(T):
                        valu(h, "%s %s, %s, %s" % (OPS[op], vr(V0 + l * T + j), vr(V0 + FO + j),
                                                   vr(V0 + FO + dl * T + j)))
                    epilogue(h)
                    hs.append(h)
    for op in ("add", "sub", "mul"):
        for l in range(D):
            h = Handler(K["XX2"], OP_ID[op], l)    # two passes: s[l] = x[b]; s[l] = x[a] op s[l]
            prologue(h, second_index=True)
            idx_on(h, "s71", ["SRC0"])
            for j in range(T):
                valu(h, "v_mov_b32_e32 %s, %s" % (vr(V0 + l * T + j), vr(V0 + j)))
            idx_on(h, "s70", ["SRC0"])
            for j in range(T):
                r = vr(V0 + l * T + j)
                valu(h, "%s %s, %s, %s" % (OPS[op], r, vr(V0 + j), r))
            epilogue(h)
            hs.append(h)
    for op, ins in (("add", "v_add_f32_e32"), ("mul", "v_mul_f32_e32"), ("sub", "v_subrev_f32_e32")):
        for l in range(D):
            h = Handler(K["XC"], OP_ID[op], l)     # push x[a] op c
            prologue(h, const=True, index=["SRC1"])
            for j in range(T):
                valu(h, "%s %s, s72, %s" % (ins, vr(V0 + l * T + j), vr(V0 + j)))
            epilogue(h)
            hs.append(h)
    for l in range(D):
        h = Handler(K["CX"], OP_ID["sub"], l)      # push c - x[b]
        prologue(h, const=True, index=["SRC1"])
        for j in range(T):
            valu(h, "v_sub_f32_e32 %s, s72, %s" % (vr(V0 + l * T + j), vr(V0 + j)))
        epilogue(h)
        hs.append(h)
    for l in range(D):
        h = Handler(K["PUSHX"], 0, l)              # s[l] = x[a] (a lone variable, an operand of IF)
        prologue(h, index=["SRC0"])
        for j in range(T):
            valu(h, "v_mov_b32_e32 %s, %s" % (vr(V0 + l * T + j), vr(V0 + j)))
        epilogue(h)
        hs.append(h)
    h = Handler(K["PUSHC"])                        # s[l] = c; index l*T
    prologue(h, const=True, index=["DST"])
    for j in range(T):
        valu(h, "v_mov_b32_e32 %s, s72" % vr(V0 + j))
    epilogue(h)
    hs.append(h)

    for kind in ("DVV", "DVC", "DCV"):
        hs.append(div_handler(kind, T, V0))
    for op in list(CMP_OPS) + list(LOGIC_OPS):
        for kind in ("CVV", "CVC", "CCV"):
            hs.append(cmp_handler(kind, op, T, V0))
    hs.append(if_handler(T, V0))

    if mode >= 3:                      # trees only: no linear handlers
        return finish(hs, tag, V0, FO)

    # ---------------------------------------------------------------- linear
    R = LIN_REGS
    for op in ("add", "sub", "mul"):
        for d in range(R):
            for s1 in range(R):
                h = Handler(K["RR"], OP_ID[op], d, s1)   # r[d] = r[s1] op src2 (index)
                prologue(h, index=["SRC1"])
                for j in range(T):
                    valu(h, "%s %s, %s, %s" % (OPS[op], vr(V0 + d * T + j), vr(V0 + s1 * T + j), vr(V0 + j)))
                epilogue(h)
                hs.append(h)
    for d in range(R):
        for s2 in range(R):
            h = Handler(K["XR"], OP_ID["sub"], d, s2)    # r[d] = src1 (index) - r[s2]
            prologue(h, index=["SRC0"])
            for j in range(T):
                valu(h, "v_sub_f32_e32 %s, %s, %s" % (vr(V0 + d * T + j), vr(V0 + j), vr(V0 + s2 * T + j)))
            epilogue(h)
            hs.append(h)
    for op in ("add", "sub", "mul"):
        for d in range(R):
            h = Handler(K["FF"], OP_ID[op], d)           # r[d] = src2; r[d] = src1 op r[d]
            prologue(h, second_index=True)
            idx_on(h, "s71", ["SRC0"])
            for j in range(T):
                valu(h, "v_mov_b32_e32 %s, %s" % (vr(V0 + d * T + j), vr(V0 + j)))
            idx_on(h, "s70", ["SRC0"])
            for j in range(T):
                r = vr(V0 + d * T + j)
                valu(h, "%s %s, %s, %s" % (OPS[op], r, vr(V0 + j), r))
            epilogue(h)
            hs.append(h)
    for op in ("add", "sub", "mul"):
        for d in range(R):
            h = Handler(K["CR"], OP_ID[op], d)           # r[d] = c op src (index)
            prologue(h, const=True, index=["SRC1"])
            for j in range(T):
                valu(h, "%s %s, s72, %s" % (OPS[op], vr(V0 + d * T + j), vr(V0 + j)))
            epilogue(h)
            hs.append(h)
    for d in range(R):
        h = Handler(K["RC"], OP_ID["sub"], d)            # r[d] = src (index) - c
        prologue(h, const=True, index=["SRC1"])
        for j in range(T):
            valu(h, "v_subrev_f32_e32 %s, s72, %s" % (vr(V0 + d * T + j), vr(V0 + j)))
        epilogue(h)
        hs.append(h)
    for d in range(R):
        h = Handler(K["MOVC"], 0, d)                     # r[d] = c
        prologue(h, const=True, index="off")
        for j in range(T):
            valu(h, "v_mov_b32_e32 %s, s72" % vr(V0 + d * T + j))
        epilogue(h)
        hs.append(h)
    for d in range(R):
        h = Handler(K["MOVX"], 0, d)                     # r[d] = src (index)
        prologue(h, index=["SRC0"])
        for j in range(T):
            valu(h, "v_mov_b32_e32 %s, %s" % (vr(V0 + d * T + j), vr(V0 + j)))
        epilogue(h)
        hs.append(h)

    return finish(hs, tag, V0, FO)


def div_handler(kind, T, V0):
    """Protected division in the core: d = |b| < 1e-6f ? 1 : a / b for the
    T slots, a and b at offsets (or the constant), d at a third offset, all
    in the exit's payload layout (byte 0 a, byte 1 b, byte 2 d).

    The quotient is the correctly rounded IEEE one, by the sequence the
    compiler emits for a binary32 division with denormals kept: scale
    operands (v_div_scale), reciprocal, two Newton-Raphson refinements of it
    and of the quotient with fused multiply-adds, the scaled fused add
    (v_div_fmas, whose scale flag is vcc) and the special-case fix-up
    (v_div_fixup).  Its dependent reads keep the compiler's spacing: one
    instruction between the reciprocal and its first use, six between the
    vcc write and v_div_fmas, two wait states between the compare's vcc
    write and the select that reads it.  Operands are copied out of the index range
    slot by slot (the index mode offsets every VGPR of the enabled fields,
    so the arithmetic runs with it off), and the select writes the result
    through the destination index."""
    a_const, b_const = kind == "DCV", kind == "DVC"
    tA, tB, tD, tR, tN, tE, tF = (vr(V0 - DIV_TMP + k) for k in range(DIV_TMP))

    def body(A, B, Dx, C):
        L = ["s_mov_b32 s80, 0x%x" % DIV_THRESHOLD]
        if a_const or b_const:
            L.append("s_set_gpr_idx_off")
            L.append("v_mov_b32_e32 %s, %s" % (tA if a_const else tB, C))
        for j in range(T):
            if not a_const:
                L.append("s_set_gpr_idx_on %s, gpr_idx(SRC0)" % A)
                L.append("v_mov_b32_e32 %s, %s" % (tA, vr(V0 + j)))
            if not b_const:
                L.append("s_set_gpr_idx_on %s, gpr_idx(SRC0)" % B)
                L.append("v_mov_b32_e32 %s, %s" % (tB, vr(V0 + j)))
            L.append("s_set_gpr_idx_off")
            L += ["v_div_scale_f32 %s, vcc, %s, %s, %s" % (tD, tB, tB, tA),
                  "v_rcp_f32_e32 %s, %s" % (tR, tD),
                  "v_div_scale_f32 %s, vcc, %s, %s, %s" % (tN, tA, tB, tA),
                  "v_fma_f32 %s, -%s, %s, 1.0" % (tE, tD, tR),
                  "v_fmac_f32_e32 %s, %s, %s" % (tR, tE, tR),
                  "v_mul_f32_e32 %s, %s, %s" % (tE, tN, tR),
                  "v_fma_f32 %s, -%s, %s, %s" % (tF, tD, tE, tN),
                  "v_fmac_f32_e32 %s, %s, %s" % (tE, tF, tR),
                  "v_fma_f32 %s, -%s, %s, %s" % (tD, tD, tE, tN),
                  "v_div_fmas_f32 %s, %s, %s, %s" % (tD, tD, tR, tE),
                  "v_div_fixup_f32 %s, %s, %s, %s" % (tD, tD, tB, tA),
                  # vcc = |b| >= 1e-6f or b is NaN: keep the quotient, else 1
                  "v_cmp_nlt_f32_e64 vcc, |%s|, s80" % tB,
                  # a vector write of a mask register is read as a lane mask two wait states later at the earliest
                  "s_nop 1",
                  "s_set_gpr_idx_on %s, gpr_idx(DST)" % Dx,
                  "v_cndmask_b32_e32 %s, 1.0, %s, vcc" % (vr(V0 + j), tD)]
        return L

    h = Handler(K[kind], 3)
    # phase A: own record in s[64:67], the next one already in s[68:71]
    la = ["s_lshr_b32 s74, s66, 8", "s_lshr_b32 s79, s66, 16"] + body("s66", "s74", "s79", "s67")
    la += ["s_add_u32 s62, s62, 16", "s_setpc_b64 s[68:69]"]
    # phase B: own record in s[68:71], saved before the load of the next two
    lb = ["s_mov_b32 s73, s70", "s_lshr_b32 s74, s70, 8", "s_lshr_b32 s79, s70, 16", "s_mov_b32 s72, s71",
          "s_add_u32 s62, s62, 16", "s_load_dwordx8 s[64:71], s[60:61], s62"] + body("s73", "s74", "s79", "s72")
    lb += ["s_waitcnt lgkmcnt(0)", "s_setpc_b64 s[64:65]"]
    h.phases = (la, lb)
    return h


# The classification functions in the core: >, <, == give 1 or 0 (an ordered
# compare: false with a NaN); AND and OR test operands for != 0 (a NaN is
# non-zero); IF(a, b, c) = a != 0 ? b : c.  Operand ids as the tree opcodes.
CMP_OPS = {12: "gt", 13: "lt", 14: "eq"}
CMP_SWAP = {"gt": "lt", "lt": "gt", "eq": "eq"}      # c op x  ==  x swap(op) c
LOGIC_OPS = {8: "s_and_b64", 9: "s_or_b64"}
IF_KIND = "IF3"


def phases_of(h, body, n_idx):
    """Both phases of a handler whose body takes its index registers (A, B,
    D[, C]) and the constant register.  Phase A finds its record in s[64:67]
    (the next one is already in s[68:71]); phase B saves what it needs from
    s[68:71] before loading the next two records over s[64:71]."""
    if n_idx == 3:
        la = ["s_lshr_b32 s74, s66, 8", "s_lshr_b32 s79, s66, 16"] + body("s66", "s74", "s79", "s67", None)
        lb = ["s_mov_b32 s73, s70", "s_lshr_b32 s74, s70, 8", "s_lshr_b32 s79, s70, 16", "s_mov_b32 s72, s71"]
        regs_b = ("s73", "s74", "s79", "s72", None)
    else:
        la = ["s_lshr_b32 s74, s66, 8", "s_lshr_b32 s73, s66, 16", "s_lshr_b32 s79, s66, 24"] + \
            body("s66", "s74", "s79", None, "s73")
        lb = ["s_mov_b32 s73, s70", "s_lshr_b32 s74, s70, 8", "s_lshr_b32 s72, s70, 16", "s_lshr_b32 s79, s70, 24"]
        regs_b = ("s73", "s74", "s79", None, "s72")
    la += ["s_add_u32 s62, s62, 16", "s_setpc_b64 s[68:69]"]
    lb += ["s_add_u32 s62, s62, 16", "s_load_dwordx8 s[64:71], s[60:61], s62"] + body(*regs_b)
    lb += ["s_waitcnt lgkmcnt(0)", "s_setpc_b64 s[64:65]"]
    h.phases = (la, lb)
    return h


def cmp_handler(kind, op, T, V0):
    """d = a op b for op in >, <, ==, AND, OR (1 or 0 per slot), a and b at
    two offsets (CVV) or one of them the record's constant (CVC: b, CCV: a),
    d at a third; the payload is the exit's layout.  A compare writes vcc
    (AND and OR first write the first operand's test to s[80:81] and combine
    them); a select through the destination index writes the result, two wait
    states after the mask is written."""
    a_const, b_const = kind == "CCV", kind == "CVC"
    tB = vr(V0 - DIV_TMP)
    name = CMP_OPS.get(op)

    def body(A, B, Dx, C, _):
        L = []
        if name is None and (a_const or b_const):
            # the constant's truth is the same in every lane
            L += ["v_cmp_neq_f32_e64 s[80:81], 0, %s" % C]
        for j in range(T):
            if name is not None:
                if a_const:          # c op b
                    L += ["s_set_gpr_idx_on %s, gpr_idx(SRC1)" % B,
                          "v_cmp_%s_f32_e32 vcc, %s, %s" % (name, C, vr(V0 + j))]
                elif b_const:        # a op c  ==  c swap(op) a
                    L += ["s_set_gpr_idx_on %s, gpr_idx(SRC1)" % A,
                          "v_cmp_%s_f32_e32 vcc, %s, %s" % (CMP_SWAP[name], C, vr(V0 + j))]
                else:                # b copied out, a through the index
                    L += ["s_set_gpr_idx_on %s, gpr_idx(SRC0)" % B,
                          "v_mov_b32_e32 %s, %s" % (tB, vr(V0 + j)),
                          "s_set_gpr_idx_on %s, gpr_idx(SRC0)" % A,
                          "v_cmp_%s_f32_e32 vcc, %s, %s" % (name, vr(V0 + j), tB)]
            else:
                if not (a_const or b_const):
                    L += ["s_set_gpr_idx_on %s, gpr_idx(SRC1)" % A,
                          "v_cmp_neq_f32_e64 s[80:81], 0, %s" % vr(V0 + j)]
                L += ["s_set_gpr_idx_on %s, gpr_idx(SRC1)" % (A if b_const else B),
                      "v_cmp_neq_f32_e32 vcc, 0, %s" % vr(V0 + j),
                      "s_nop 1",
                      "%s vcc, vcc, s[80:81]" % LOGIC_OPS[op]]
            L += ["s_nop 1",
                  "s_set_gpr_idx_on %s, gpr_idx(DST)" % Dx,
                  "v_cndmask_b32_e64 %s, 0, 1.0, vcc" % vr(V0 + j)]
        return L

    return phases_of(Handler(K[kind], op), body, 3)


def if_handler(T, V0):
    """IF(a, b, c) = a != 0 ? b : c (a NaN is non-zero) over three offsets,
    the result to a fourth (payload bytes 0-3: a, b, c, d)."""
    tB, tC = vr(V0 - DIV_TMP), vr(V0 - DIV_TMP + 1)

    def body(A, B, Dx, _, Cx):
        L = []
        for j in range(T):
            L += ["s_set_gpr_idx_on %s, gpr_idx(SRC0)" % B,
                  "v_mov_b32_e32 %s, %s" % (tB, vr(V0 + j)),
                  "s_set_gpr_idx_on %s, gpr_idx(SRC0)" % Cx,
                  "v_mov_b32_e32 %s, %s" % (tC, vr(V0 + j)),
                  "s_set_gpr_idx_on %s, gpr_idx(SRC1)" % A,
                  "v_cmp_neq_f32_e32 vcc, 0, %s" % vr(V0 + j),
                  "s_nop 1",
                  "s_set_gpr_idx_on %s, gpr_idx(DST)" % Dx,
                  "v_cndmask_b32_e32 %s, %s, %s, vcc" % (vr(V0 + j), tC, tB)]
        return L

    return phases_of(Handler(K[IF_KIND], 15), body, 4)


def bool_handlers(hs, T, D, V0, FO, prologue, idx_on, epilogue, valu):
    """Handlers of the Boolean function set.  Every function is symmetric, so
    only the forms with the stack (or first) operand on the left exist: SS,
    SX, XX2 (two features, two passes) and PUSHX.  Each function is one
    vector instruction per slot; the index mode offsets the same sources and
    destination in every encoding."""
    for op in BOOL_OPS:
        h = Handler(K["SS"], BOOL_ID[op])           # s[h-2] = s[h-2] op s[h-1]; index (h-2)*T
        prologue(h, index=["SRC0", "SRC1", "DST"])
        for j in range(T):
            valu(h, bool_op(op, vr(V0 + j), vr(V0 + j), vr(V0 + T + j)))
        epilogue(h)
        hs.append(h)
    for op in BOOL_OPS:
        for l in range(D):
            h = Handler(K["SX"], BOOL_ID[op], l)    # s[l] = s[l] op x[b]; index = feature offset
            prologue(h, index=["SRC1"])
            for j in range(T):
                r = vr(V0 + l * T + j)
                valu(h, bool_op(op, r, r, vr(V0 + j)))
            epilogue(h)
            hs.append(h)
    for op in BOOL_OPS:
        for l in range(D):
            h = Handler(K["XX2"], BOOL_ID[op], l)   # s[l] = x[b]; s[l] = x[a] op s[l]
            prologue(h, second_index=True)
            idx_on(h, "s71", ["SRC0"])
            for j in range(T):
                valu(h, "v_mov_b32_e32 %s, %s" % (vr(V0 + l * T + j), vr(V0 + j)))
            idx_on(h, "s70", ["SRC0"])
            for j in range(T):
                r = vr(V0 + l * T + j)
                valu(h, bool_op(op, r, vr(V0 + j), r))
            epilogue(h)
            hs.append(h)
    h = Handler(K["PUSHX"])                         # s[0] = x[a] (a program that is one variable)
    prologue(h, index=["SRC0"])
    for j in range(T):
        valu(h, "v_mov_b32_e32 %s, %s" % (vr(V0 + j), vr(V0 + j)))
    epilogue(h)
    hs.append(h)


def finish(hs, tag, V0, FO):
    """Both phases of every handler, laid out in 64-byte slots."""
    hs = [phase_a(h, tag) for h in hs] + [phase_b(h, tag) for h in hs]
    slot = 0
    for h in hs:
        h.slot = slot
        slot += (h.size + SLOT - 1) // SLOT
    return tag, V0, FO, hs, slot


# Two copies of every handler.  Records are fetched two at a time: a phase-B
# handler (its own record in s[68:71]) loads the next two records into
# s[64:71] with one s_load_dwordx8, works, waits, and jumps to the next
# instruction's phase-A handler; a phase-A handler (its record in s[64:67],
# the next one already in s[68:71]) works and jumps on without loading or
# waiting.  So only every second instruction waits for the scalar cache.
# The host gives instructions alternating phases, A first after every entry
# into the core (program start, return from an exit), which loads the first
# two records itself.  The handlers are written once (as for a single record
# in s[64:67], constant copied to s72, indexes in s66/s70/s71); these
# functions rewrite them for each phase.
PHASE_B = 0x80


def _copy(h, kind):
    c = Handler(kind, h.op, h.p1, h.p2)
    return c


def phase_a(h, tag):
    c = _copy(h, h.kind)
    if h.phases:
        for x in h.phases[0]:
            c.emit(x, insn_bytes(x))
        return c
    if h.kind == K["EXIT"]:
        for x in h.lines:
            c.emit(x, 4)
        return c
    body = []
    for x in h.lines:
        if x == "s_mov_b32 s72, s67" or x == "s_mov_b32 s70, s66" or x.startswith("s_add_u32 s62") \
                or x.startswith("s_load_dwordx4") or x.startswith("s_waitcnt") or x.startswith("s_setpc"):
            continue
        x = x.replace("s_lshr_b32 s71, s66, 8", "s_lshr_b32 s74, s66, 8")
        x = x.replace("s_set_gpr_idx_on s70,", "s_set_gpr_idx_on s66,").replace("s_set_gpr_idx_on s71,", "s_set_gpr_idx_on s74,")
        x = x.replace("s72", "s67")
        body.append(x)
    for x in body:
        c.emit(x, insn_bytes(x))
    c.emit("s_add_u32 s62, s62, 16", 4)
    c.emit("s_setpc_b64 s[68:69]", 4)
    return c


def phase_b(h, tag):
    c = _copy(h, h.kind | PHASE_B)
    if h.phases:
        for x in h.phases[1]:
            c.emit(x, insn_bytes(x))
        return c
    if h.kind == K["EXIT"]:
        c.emit("s_set_gpr_idx_off", 4)
        c.emit("s_mov_b32 s66, s70", 4)
        c.emit("s_mov_b32 s67, s71", 4)
        c.emit("s_branch .Lgpx_end_%s" % tag, 4)
        return c
    for x in h.lines:
        if x == "s_mov_b32 s72, s67":
            x = "s_mov_b32 s72, s71"
        elif x == "s_mov_b32 s70, s66":
            x = "s_mov_b32 s73, s70"
        elif x == "s_lshr_b32 s71, s66, 8":
            x = "s_lshr_b32 s74, s70, 8"
        elif x.startswith("s_load_dwordx4"):
            x = "s_load_dwordx8 s[64:71], s[60:61], s62"
        elif x.startswith("s_set_gpr_idx_on s66,"):
            x = x.replace("s_set_gpr_idx_on s66,", "s_set_gpr_idx_on s70,")
        elif x.startswith("s_set_gpr_idx_on s70,"):
            x = x.replace("s_set_gpr_idx_on s70,", "s_set_gpr_idx_on s73,")
        elif x.startswith("s_set_gpr_idx_on s71,"):
            x = x.replace("s_set_gpr_idx_on s71,", "s_set_gpr_idx_on s74,")
        c.emit(x, insn_bytes(x))
    return c


def asm_text(T, D, NF, tag, hs):
    L = []
    L.append("s_getpc_b64 s[76:77]")
    L.append(".Lgpx_pc_%s:" % tag)
    L.append("s_cmp_eq_u32 s63, 0")
    L.append("s_cbranch_scc1 .Lgpx_run_%s" % tag)
    L.append("s_add_u32 s76, s76, .Lgpx_table_%s-.Lgpx_pc_%s" % (tag, tag))
    L.append("s_addc_u32 s77, s77, 0")
    L.append("s_branch .Lgpx_end_%s" % tag)
    L.append(".Lgpx_run_%s:" % tag)
    # Burst-load the program's remaining 64-byte lines (from the current
    # record's line up to byte offset s75) into the scalar cache, up to s78
    # loads in flight, so the handlers' record loads then hit.  s75 = 0 skips
    # it (re-entry after an exit).  s76 only receives data; every load is
    # waited for before the first handler runs.
    L.append("s_and_b32 s73, s62, 0xffffffc0")
    L.append("s_mov_b32 s74, 0")
    L.append(".Lgpx_pf_%s:" % tag)
    L.append("s_cmp_lt_u32 s73, s75")
    L.append("s_cbranch_scc0 .Lgpx_pfdone_%s" % tag)
    L.append("s_load_dword s76, s[60:61], s73")
    L.append("s_add_u32 s73, s73, 64")
    L.append("s_add_u32 s74, s74, 1")
    L.append("s_cmp_lt_u32 s74, s78")
    L.append("s_cbranch_scc1 .Lgpx_pf_%s" % tag)
    L.append("s_waitcnt lgkmcnt(0)")
    L.append("s_mov_b32 s74, 0")
    L.append("s_branch .Lgpx_pf_%s" % tag)
    L.append(".Lgpx_pfdone_%s:" % tag)
    L.append("s_load_dwordx8 s[64:71], s[60:61], s62")   # this record and the next: phase A
    L.append("s_waitcnt lgkmcnt(0)")
    L.append("s_setpc_b64 s[64:65]")
    L.append(".p2align %d" % (SLOT.bit_length() - 1))
    L.append(".Lgpx_table_%s:" % tag)
    for i, h in enumerate(hs):
        lab = ".Lgpx_h%d_%s" % (i, tag)
        L.append("%s:" % lab)
        # the host addresses handlers by slot: check the slot arithmetic
        L.append(".if (%s - .Lgpx_table_%s) != %d" % (lab, tag, h.slot * SLOT))
        L.append('.error \\"gpx handler %d misplaced\\"' % i)
        L.append(".endif")
        L.extend(h.lines)
        # pad to the slot boundary (never executed: every handler ends in a jump)
        pad = (-h.size) % SLOT
        L.extend(["s_nop 0"] * (pad // 4))
    L.append(".Lgpx_end_%s:" % tag)
    return "\\n\\t".join(L)


def gather_scatter(T, V0):
    """C++ helpers moving T slots between compiler VGPRs and the core's range."""
    out = []
    tv = "%d, %d" % (T, V0)
    outs = ", ".join('"=v"(v[%d])' % j for j in range(T))
    movs = "".join("v_mov_b32_e32 %%%d, %s\\n\\t" % (j, vr(V0 + j)) for j in range(T))
    out.append("template <> __device__ __forceinline__ void core_gather<%s>(uint32_t off, float (&v)[%d]) {" % (tv, T))
    out.append("#ifdef __HIP_DEVICE_COMPILE__")
    out.append('    asm volatile("s_set_gpr_idx_on %%%d, gpr_idx(SRC0)\\n\\t%ss_set_gpr_idx_off" : %s : "s"(off) : "m0");'
               % (T, movs, outs))
    out.append("#endif")
    out.append("}")
    # gather, or broadcast the constant when use_const is nonzero: one scalar
    # branch inside the asm, so the compiler cannot run both paths
    cmovs = "".join("v_mov_b32_e32 %%%d, %%%d\\n\\t" % (j, T + 2) for j in range(T))
    gmovs = "".join("v_mov_b32_e32 %%%d, %s\\n\\t" % (j, vr(V0 + j)) for j in range(T))
    out.append("template <> __device__ __forceinline__ void core_gather_or_const<%s>(uint32_t off, uint32_t use_const, "
               "uint32_t cbits, float (&v)[%d]) {" % (tv, T))
    out.append("#ifdef __HIP_DEVICE_COMPILE__")
    out.append('    asm volatile("s_cmp_eq_u32 %%%d, 0\\n\\ts_cbranch_scc1 1f\\n\\t%ss_branch 2f\\n1:\\n\\t'
               's_set_gpr_idx_on %%%d, gpr_idx(SRC0)\\n\\t%ss_set_gpr_idx_off\\n2:" : %s : "s"(off), "s"(use_const), '
               '"s"(cbits) : "m0", "scc");' % (T + 1, cmovs, T, gmovs, outs))
    out.append("#endif")
    out.append("}")
    ins = ", ".join('"v"(v[%d])' % j for j in range(T))
    movs = "".join("v_mov_b32_e32 %s, %%%d\\n\\t" % (vr(V0 + j), j + 1) for j in range(T))
    out.append("template <> __device__ __forceinline__ void core_scatter<%s>(uint32_t off, const float (&v)[%d]) {"
               % (tv, T))
    out.append("#ifdef __HIP_DEVICE_COMPILE__")
    out.append('    asm volatile("s_set_gpr_idx_on %%0, gpr_idx(DST)\\n\\t%ss_set_gpr_idx_off" : : "s"(off), %s : "m0");'
               % (movs, ins))
    out.append("#endif")
    out.append("}")
    return "\n".join(out)


def main(out_dir):
    os.makedirs(out_dir, exist_ok=True)
    lines = ["// Generated by gen_core.py -- do not edit.", "#pragma once", ""]
    lines.append("#define GPX_LIN_REGS %d" % LIN_REGS)
    lines.append("#define GPX_SLOT %d" % SLOT)
    lines.append("enum CoreKind {" + ", ".join("CK_%s = %d" % (k, i) for i, k in enumerate(KINDS)) + "};")
    lines.append("")
    lines.append("#define GPX_CORE_VARIANTS(X) \\")
    lines.append(" \\\n".join("    X(%d, %d, %d, %d, %d)" % v for v in VARIANTS))
    lines.append("")
    clob_s = ", ".join('"s%d"' % n for n in (63, 64, 65, 66, 67, 70, 71, 72, 76, 77))
    lines.append("template <int T, int D, int NF, int V0, int K> struct Core;   // K: 0 arithmetic, 2 Boolean, 3 trees only")
    lines.append("template <int T, int V0> __device__ void core_gather(uint32_t off, float (&v)[T]);")
    lines.append("template <int T, int V0> __device__ void core_scatter(uint32_t off, const float (&v)[T]);")
    lines.append("template <int T, int V0> __device__ void core_gather_or_const(uint32_t off, uint32_t use_const, "
                 "uint32_t cbits, float (&v)[T]);")
    for T, V0 in sorted(set((v[0], v[3]) for v in VARIANTS)):
        lines.append(gather_scatter(T, V0))
    host = []
    seen = {}
    for (T, D, NF, NCV, AR) in VARIANTS:
        B = AR == 2
        core = (T, D, NF, NCV, {1: 0, 4: 3}.get(AR, AR))   # modes 0 and 1 share a core, so do 3 and 4
        if core in seen:
            host.append((T, D, NF, NCV, AR) + seen[core])
            continue
        tag, V0, FO, hs, nslots = gen_variant(T, D, NF, NCV, AR)
        seen[core] = (tag, hs, nslots)
        text = asm_text(T, D, NF, tag, hs)
        clob_v = ", ".join('"%s"' % vr(n) for n in range(NCV, NCV + FO + NF * T))
        if AR != 2:    # the division and classification handlers' temporaries, flags, indexes and threshold
            clob_v += ", " + ", ".join('"%s"' % vr(n) for n in range(NCV - DIV_TMP, NCV)) + \
                ', "vcc", "s79", "s80", "s81"'
            assert NCV - DIV_TMP >= 24
        assert NCV + FO + NF * T <= 256
        lines.append("template <> struct Core<%d, %d, %d, %d, %d> {" % (T, D, NF, NCV, core[4]))
        lines.append("    // run from byte offset `off` until an exit; returns the exit's payload and constant")
        lines.append("    // pf_end: byte offset where the program ends (its code is first burst-loaded into the")
        lines.append("    // scalar cache, `burst` loads in flight at a time), or 0")
        lines.append("    static __device__ __forceinline__ void run(uint64_t base, uint32_t& off, uint32_t& pay,"
                     " uint32_t& cst, uint32_t probe, uint32_t pf_end, uint32_t burst, uint64_t& table) {")
        lines.append("#ifdef __HIP_DEVICE_COMPILE__")
        lines.append('        asm volatile("%s"' % text)
        lines.append('            : "+{s62}"(off), "={s66}"(pay), "={s67}"(cst), "={s[76:77]}"(table)')
        lines.append('            : "{s[60:61]}"(base), "{s63}"(probe), "{s75}"(pf_end), "{s78}"(burst)')
        lines.append('            : %s, "s64", "s65", "s68", "s69", "s70", "s71", "s72", "s73", "s74", "scc", "m0",'
                     ' "memory");' % clob_v)
        lines.append("#endif")
        lines.append("    }")
        lines.append("};")
        host.append((T, D, NF, NCV, AR, tag, hs, nslots))
    lines.append("")
    lines.append("struct CoreHandlerKey { uint8_t kind, op; int8_t p1, p2; };")
    done = set()
    for (T, D, NF, NCV, AR, tag, hs, nslots) in host:
        if tag in done:
            continue
        done.add(tag)
        lines.append("static const CoreHandlerKey kCoreKeys_%s[] = {" % tag)
        lines.append("    " + ", ".join("{%d,%d,%d,%d}" % (h.kind, h.op, h.p1, h.p2) for h in hs))
        lines.append("};")
        lines.append("static const uint16_t kCoreSlots_%s[] = {" % tag)
        lines.append("    " + ", ".join(str(h.slot) for h in hs))
        lines.append("};")
    lines.append("struct CoreVariantDesc { int t, d, nf, ncv, arith; const CoreHandlerKey* keys; const uint16_t* slots; "
                 "int n; int table_bytes; };")
    lines.append("static const CoreVariantDesc kCoreVariants[] = {")
    for (T, D, NF, NCV, AR, tag, hs, nslots) in host:
        lines.append("    {%d, %d, %d, %d, %d, kCoreKeys_%s, kCoreSlots_%s, %d, %d}," % (T, D, NF, NCV, AR, tag, tag, len(hs),
                                                                                    nslots * SLOT))
    lines.append("};")
    path = os.path.join(out_dir, "core_gen.inc")
    write_if_changed(path, "\n".join(lines) + "\n")
    # one translation unit per kernel variant, and the launch table
    disp = ["// Generated by gen_core.py -- do not edit.", "#pragma once", "",
            "typedef hipError_t (*CoreLaunchFn)(const CoreArgs&, uint32_t, hipStream_t);",
            "typedef int (*CoreOccupancyFn)();"]
    for (T, D, NF, NCV, AR, tag, hs, nslots) in host:
        name = vname((T, D, NF, NCV, AR))
        disp.append("hipError_t core_launch_%s(const CoreArgs& a, uint32_t blocks, hipStream_t s);" % name)
        disp.append("int core_occupancy_%s();" % name)
        tu = ["// Generated by gen_core.py -- do not edit.  Kernel variant %s." % tag,
              '#include "core_body.h"', "", "namespace gpx {",
              "GPX_KERNEL(%d, %d, %d, %d, %d, %s)" % (T, D, NF, NCV, AR, name), "",
              "hipError_t core_launch_%s(const CoreArgs& a, uint32_t blocks, hipStream_t s) {" % name,
              "    hipLaunchKernelGGL(k_core_%s, dim3(blocks), dim3(256), 0, s, a);" % name,
              "    return hipGetLastError();", "}", "",
              "int core_occupancy_%s() {" % name,
              "    int n = 0;",
              "    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_core_%s, 256, 0) != hipSuccess) n = 1;" % name,
              "    return n;", "}", "}  // namespace gpx", ""]
        write_if_changed(os.path.join(out_dir, "core_v_%s.hip" % name), "\n".join(tu))
    names = [vname(h[:5]) for h in host]
    disp.append("static const CoreLaunchFn kCoreLaunch[] = {%s};" % ", ".join("core_launch_" + n for n in names))
    disp.append("static const CoreOccupancyFn kCoreOccupancy[] = {%s};"
                % ", ".join("core_occupancy_" + n for n in names))
    write_if_changed(os.path.join(out_dir, "core_dispatch.inc"), "\n".join(disp) + "\n")
    for (T, D, NF, NCV, AR, tag, hs, nslots) in host:
        print("%s%s: %d handlers, %d slots (%d KiB)" % (tag, "a" if AR == 1 else "", len(hs), nslots, nslots * SLOT // 1024))
    return path


def variant_sources():
    """File names of the generated per-variant translation units."""
    return ["core_v_%s.hip" % vname(v) for v in VARIANTS]


def write_if_changed(path, text):
    """Write text unless the file already holds it (keeps mtimes for incremental builds)."""
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path + ".tmp", "w") as f:
        f.write(text)
    os.replace(path + ".tmp", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else ".")
