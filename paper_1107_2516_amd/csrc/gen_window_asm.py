#!/usr/bin/env python3
"""Generate dd_window_asm.inc: the register-window inner step of the FP32
de-dispersion kernel, as gfx950 inline assembly.

    python gen_window_asm.py > dd_window_asm.inc

Why assembly: a lane owns K consecutive output samples of DW trial DMs.  For
one channel, the samples those DMs need are K-long runs of the staged channel
window at wave-uniform offsets r_j.  The lane loads one register window of
WMAX consecutive samples and serves every DM whose run fits in it, using
VGPR-relative addressing (s_set_gpr_idx_on with the SRC0 mode) so that each
add reads window[r_j - start + k] with a run-time, wave-uniform offset and no
extra instruction.  The window has to sit in fixed, consecutive VGPRs for that
addressing, which only inline assembly can guarantee; it is declared clobbered
and lives only inside one asm statement.

Per DM j the block:
  * reloads the window (WMAX/4 ds_read_b128) when r_j falls outside the
    current one (start aligned down to 4 samples),
  * runs K v_add_f32 with SRC0 indexed by r_j - start.
After the first DM the step issues the scalar load of the next channel's
shifts (`next`, returned in `rn`); it completes behind the remaining DMs.
"""
import sys

CONFIGS = [
    # name, DMs per wave, samples per lane, window registers, waves per SIMD
    ("f32_d8_k20_w56", 8, 20, 56, 2),
    ("f32_d8_k12_w48", 8, 12, 48, 3),
    ("f32_d4_k20_w56", 4, 20, 56, 3),
    ("f32_d6_k12_w64", 6, 12, 64, 3),
    ("f32_d4_k12_w40", 4, 12, 40, 4),
]


def vgpr_budget(occ):
    """VGPRs per lane available to a wave when `occ` waves share a SIMD
    (512 per lane, allocated in granules of 8)."""
    return min(256, (512 // occ) // 8 * 8)


def prefetch_decl(dw):
    """Locals of a channel step, including the SGPR tuple that receives the
    next channel's shifts."""
    vec = "int4v" if dw <= 4 else "int8v"
    return ["  int ws, ix, tb;", "  unsigned va;", f"  {vec} nv;"]


def prefetch_issue(dw):
    """The next channel's shifts are loaded once the first DM's window has
    arrived, so the channel's only mandatory LDS wait does not also wait for
    this scalar load; the step ends with a wait for it."""
    op = "s_load_dwordx4" if dw <= 4 else "s_load_dwordx8"
    return f'      "{op} %[rn], %[tp], 0\\n"'


def prefetch_store(dw):
    return [f"  for (int i = 0; i < {dw}; i++) rn[i] = nv[i];"]


def gen(name, dw, k, wmax, occ):
    assert k % 4 == 0 and wmax % 4 == 0 and wmax >= k + 4
    # the window sits at the top of the wave's VGPR budget so the kernel's
    # register count (and so its occupancy) is not raised by it
    wb = vgpr_budget(occ) - wmax
    out = []
    out.append(f"// {name}: DW={dw} K={k} WMAX={wmax} OCC={occ}, window v{wb}..v{wb + wmax - 1}")
    out.append(f"#define DD_{name.upper()}_DW {dw}")
    out.append(f"#define DD_{name.upper()}_K {k}")
    out.append(f"#define DD_{name.upper()}_WMAX {wmax}")
    out.append(f"__device__ __forceinline__ void dd_{name}_channel(float* acc, const int* r, unsigned addr, const int32_t* next, int* rn) {{")
    out += prefetch_decl(dw)
    out.append("  asm volatile(")
    out.append('      "s_mov_b32 %[ws], 0x80000000\\n"')
    for j in range(dw):
        out.append(f'      "s_sub_u32 %[ix], %[r{j}], %[ws]\\n"')
        out.append(f'      "s_cmp_gt_u32 %[ix], {wmax - k}\\n"')
        out.append(f'      "s_cbranch_scc0 .Lkeep_%=_{j}\\n"')
        out.append(f'      "s_and_b32 %[ws], %[r{j}], -4\\n"')
        out.append(f'      "s_sub_u32 %[ix], %[r{j}], %[ws]\\n"')
        out.append('      "s_lshl_b32 %[tb], %[ws], 2\\n"')
        out.append('      "v_add_u32 %[va], %[tb], %[addr]\\n"')
        for i in range(wmax // 4):
            off = f" offset:{16 * i}" if i else ""
            out.append(f'      "ds_read_b128 v[{wb + 4 * i}:{wb + 4 * i + 3}], %[va]{off}\\n"')
        out.append('      "s_waitcnt lgkmcnt(0)\\n"')
        out.append(f'      ".Lkeep_%=_{j}:\\n"')
        out.append('      "s_set_gpr_idx_on %[ix], gpr_idx(SRC0)\\n"')
        out.append('      "s_nop 0\\n"')
        for kk in range(k):
            out.append(f'      "v_add_f32 %[a{j}_{kk}], v{wb + kk}, %[a{j}_{kk}]\\n"')
        out.append('      "s_set_gpr_idx_off\\n"')
        if j == 0:
            out.append(prefetch_issue(dw))
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[ws] "=&s"(ws)', '[ix] "=&s"(ix)', '[tb] "=&s"(tb)', '[va] "=&v"(va)',
             '[rn] "=&s"(nv)']
    ins = ['[addr] "v"(addr)', '[tp] "s"(next)'] + [f'[r{j}] "s"(r[{j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)] + ['"m0"', '"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out += prefetch_store(dw)
    out.append("}")
    return "\n".join(out)


def gen_sched(name, dw, k, wmax, occ):
    """Scheduled flavour: the host has already run the window logic (plan
    table "wintab"), so each DM's table entry holds its window index ix
    (bits 0-7; bits 8-15 are zero), the window start for a reload (bits
    16-29), a reload flag (bit 31) and, on DM 0, whether any later DM of the
    wavefront reloads at this channel (bit 30).  DM 0 always loads the window.  When no later DM
    reloads (the common case once the shift spread of the wavefront's DMs is
    below WMAX-K), the DMs run back to back inside one indexing region, each
    switching only the index (s_set_gpr_idx_idx reads entry bits 0-7); the
    other channels take the per-DM path with a reload test on bit 31."""
    assert k % 4 == 0 and wmax % 4 == 0 and wmax >= k + 4 and wmax - k <= 255
    wb = vgpr_budget(occ) - wmax
    out = []
    out.append(f"// s_{name}: DW={dw} K={k} WMAX={wmax} OCC={occ}, window v{wb}..v{wb + wmax - 1}, "
               f"host-scheduled reloads")
    out.append(f"__device__ __forceinline__ void dd_s_{name}_channel(float* acc, const int* r, unsigned addr, const int32_t* next, int* rn) {{")
    vec = "int4v" if dw <= 4 else "int8v"
    out += ["  int tb;", "  unsigned va;", f"  {vec} nv;"]
    out.append("  asm volatile(")

    def reload(j):
        lines = [f'      "s_bfe_u32 %[tb], %[r{j}], 0xe0010\\n"',  # bits 16..29: window start
                 '      "s_lshl_b32 %[tb], %[tb], 2\\n"',
                 '      "v_add_u32 %[va], %[tb], %[addr]\\n"']
        for i in range(wmax // 4):
            off = f" offset:{16 * i}" if i else ""
            lines.append(f'      "ds_read_b128 v[{wb + 4 * i}:{wb + 4 * i + 3}], %[va]{off}\\n"')
        lines.append('      "s_waitcnt lgkmcnt(0)\\n"')
        return lines

    def adds(j):
        return [f'      "v_add_f32 %[a{j}_{kk}], v{wb + kk}, %[a{j}_{kk}]\\n"' for kk in range(k)]

    out += reload(0)
    out.append('      "s_set_gpr_idx_on %[r0], gpr_idx(SRC0)\\n"')
    out.append('      "s_nop 0\\n"')
    out += adds(0)
    out.append(prefetch_issue(dw))
    if dw > 1:
        out.append('      "s_bitcmp1_b32 %[r0], 30\\n"')
        out.append('      "s_cbranch_scc1 .Lslow_%=\\n"')
        for j in range(1, dw):
            out.append(f'      "s_set_gpr_idx_idx %[r{j}]\\n"')
            out.append('      "s_nop 0\\n"')
            out += adds(j)
        out.append('      "s_branch .Ldone_%=\\n"')
        out.append('      ".Lslow_%=:\\n"')
        for j in range(1, dw):
            out.append(f'      "s_bitcmp1_b32 %[r{j}], 31\\n"')
            out.append(f'      "s_cbranch_scc0 .Lkeep_%=_{j}\\n"')
            out.append('      "s_set_gpr_idx_off\\n"')
            out += reload(j)
            out.append(f'      "s_set_gpr_idx_on %[r{j}], gpr_idx(SRC0)\\n"')
            out.append(f'      ".Lkeep_%=_{j}:\\n"')
            out.append(f'      "s_set_gpr_idx_idx %[r{j}]\\n"')
            out.append('      "s_nop 0\\n"')
            out += adds(j)
        out.append('      ".Ldone_%=:\\n"')
    out.append('      "s_set_gpr_idx_off\\n"')
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[tb] "=&s"(tb)', '[va] "=&v"(va)', '[rn] "=&s"(nv)']
    ins = ['[addr] "v"(addr)', '[tp] "s"(next)'] + [f'[r{j}] "s"(r[{j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)] + ['"m0"', '"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out += prefetch_store(dw)
    out.append("}")
    return "\n".join(out)


JT_CONFIGS = [
    # jump-table flavour: name, DMs per wave, samples per lane, window, waves per SIMD
    ("jt_f32_d8_k20_w56", 8, 20, 56, 2),
    ("jt_f32_d8_k12_w48", 8, 12, 48, 3),
    ("jt_f32_d4_k20_w56", 4, 20, 56, 3),
]

# fixed SGPRs used for computed jumps inside the jump-table blocks
PC_LO, PC_HI, T_LO, T_HI = 88, 89, 90, 91


def gen_jt(name, dw, k, wmax, occ):
    """Jump-table flavour: instead of VGPR-relative addressing (which issues
    the adds at half rate on gfx950), each DM jumps with s_setpc_b64 into one
    of WMAX-K+1 pre-specialised blocks of K plain v_add_f32, block ix reading
    window registers ix..ix+K-1.  Every block is K+1 four-byte instructions,
    so block ix starts at table + ix*4*(K+1)."""
    assert k % 4 == 0 and wmax % 4 == 0 and wmax >= k + 4
    wb = vgpr_budget(occ) - wmax
    nv = wmax - k + 1
    bs = 4 * (k + 1)
    out = []
    out.append(f"// {name}: DW={dw} K={k} WMAX={wmax} OCC={occ}, window v{wb}..v{wb + wmax - 1}, "
               f"{nv} blocks of {bs} bytes per DM")
    out.append(f"__device__ __forceinline__ void dd_{name}_channel(float* acc, const int* r, unsigned addr, const int32_t* next, int* rn) {{")
    out += prefetch_decl(dw)
    out.append("  asm volatile(")
    out.append('      "s_mov_b32 %[ws], 0x80000000\\n"')
    out.append(f'      "s_getpc_b64 s[{PC_LO}:{PC_HI}]\\n"')
    out.append('      ".Lpc_%=:\\n"')
    for j in range(dw):
        out.append(f'      "s_sub_u32 %[ix], %[r{j}], %[ws]\\n"')
        out.append(f'      "s_cmp_gt_u32 %[ix], {wmax - k}\\n"')
        out.append(f'      "s_cbranch_scc0 .Lkeep_%=_{j}\\n"')
        out.append(f'      "s_and_b32 %[ws], %[r{j}], -4\\n"')
        out.append(f'      "s_sub_u32 %[ix], %[r{j}], %[ws]\\n"')
        out.append('      "s_lshl_b32 %[tb], %[ws], 2\\n"')
        out.append('      "v_add_u32 %[va], %[tb], %[addr]\\n"')
        for i in range(wmax // 4):
            off = f" offset:{16 * i}" if i else ""
            out.append(f'      "ds_read_b128 v[{wb + 4 * i}:{wb + 4 * i + 3}], %[va]{off}\\n"')
        out.append('      "s_waitcnt lgkmcnt(0)\\n"')
        out.append(f'      ".Lkeep_%=_{j}:\\n"')
        out.append(f'      "s_mul_i32 %[tb], %[ix], {bs}\\n"')
        out.append(f'      "s_add_u32 s{T_LO}, s{PC_LO}, %[tb]\\n"')
        out.append(f'      "s_addc_u32 s{T_HI}, s{PC_HI}, 0\\n"')
        out.append(f'      "s_add_u32 s{T_LO}, s{T_LO}, .Ltab_%=_{j}-.Lpc_%=\\n"')
        out.append(f'      "s_addc_u32 s{T_HI}, s{T_HI}, 0\\n"')
        out.append(f'      "s_setpc_b64 s[{T_LO}:{T_HI}]\\n"')
        out.append(f'      ".Ltab_%=_{j}:\\n"')
        for ix in range(nv):
            for kk in range(k):
                out.append(f'      "v_add_f32_e32 %[a{j}_{kk}], v{wb + ix + kk}, %[a{j}_{kk}]\\n"')
            out.append(f'      "s_branch .Lnext_%=_{j}\\n"')
        out.append(f'      ".Lnext_%=_{j}:\\n"')
        if j == 0:
            out.append(prefetch_issue(dw))
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[ws] "=&s"(ws)', '[ix] "=&s"(ix)', '[tb] "=&s"(tb)', '[va] "=&v"(va)',
             '[rn] "=&s"(nv)']
    ins = ['[addr] "v"(addr)', '[tp] "s"(next)'] + [f'[r{j}] "s"(r[{j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)] + [f'"s{i}"' for i in (PC_LO, PC_HI, T_LO, T_HI)]
    clob += ['"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out += prefetch_store(dw)
    out.append("}")
    return "\n".join(out)


PAIR_CONFIGS = [
    # 8-bit input as 16-bit sample pairs: name, DMs per wave, samples per lane,
    # window registers, waves per SIMD
    ("u8p_d8_k28_w84", 8, 28, 84, 2),
    ("u8p_d8_k20_w76", 8, 20, 76, 2),
    ("u8p_d8_k20_w56", 8, 20, 56, 3),
    ("u8p_d4_k28_w64", 4, 28, 64, 3),
]


def gen_pairs(name, dw, k, wmax, occ):
    """Pair flavour for 8-bit input.  The staged window holds one dword per
    sample position s: sample s in the low 16 bits and sample s+1 in the high
    16 bits.  A lane owns K consecutive outputs as K/2 accumulators, each two
    16-bit sums (outputs 2i and 2i+1), so one v_add_u32 adds two samples, and
    DM j reads window dwords ix_j + 2i.  No 16-bit lane can carry into its
    neighbour as long as the caller empties the accumulators at least every
    257 channels (257 * 255 < 2^16)."""
    assert k % 4 == 0 and wmax % 4 == 0 and wmax >= k + 4
    wb = vgpr_budget(occ) - wmax
    na = k // 2
    lim = wmax - k + 1  # largest ix with ix + 2*(na-1) inside the window
    out = []
    out.append(f"// {name}: DW={dw} K={k} WMAX={wmax} OCC={occ}, window v{wb}..v{wb + wmax - 1}")
    out.append(f"__device__ __forceinline__ void dd_{name}_channel(uint32_t* acc, const int* r, unsigned addr, const int32_t* next, int* rn) {{")
    out += prefetch_decl(dw)
    out.append("  asm volatile(")
    out.append('      "s_mov_b32 %[ws], 0x80000000\\n"')
    for j in range(dw):
        out.append(f'      "s_sub_u32 %[ix], %[r{j}], %[ws]\\n"')
        out.append(f'      "s_cmp_gt_u32 %[ix], {lim}\\n"')
        out.append(f'      "s_cbranch_scc0 .Lkeep_%=_{j}\\n"')
        out.append(f'      "s_and_b32 %[ws], %[r{j}], -4\\n"')
        out.append(f'      "s_sub_u32 %[ix], %[r{j}], %[ws]\\n"')
        out.append('      "s_lshl_b32 %[tb], %[ws], 2\\n"')
        out.append('      "v_add_u32 %[va], %[tb], %[addr]\\n"')
        for i in range(wmax // 4):
            off = f" offset:{16 * i}" if i else ""
            out.append(f'      "ds_read_b128 v[{wb + 4 * i}:{wb + 4 * i + 3}], %[va]{off}\\n"')
        out.append('      "s_waitcnt lgkmcnt(0)\\n"')
        out.append(f'      ".Lkeep_%=_{j}:\\n"')
        out.append('      "s_set_gpr_idx_on %[ix], gpr_idx(SRC0)\\n"')
        out.append('      "s_nop 0\\n"')
        for i in range(na):
            out.append(f'      "v_add_u32 %[a{j}_{i}], v{wb + 2 * i}, %[a{j}_{i}]\\n"')
        out.append('      "s_set_gpr_idx_off\\n"')
        if j == 0:
            out.append(prefetch_issue(dw))
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    outs = []
    for j in range(dw):
        for i in range(na):
            outs.append(f'[a{j}_{i}] "+v"(acc[{j * na + i}])')
    outs += ['[ws] "=&s"(ws)', '[ix] "=&s"(ix)', '[tb] "=&s"(tb)', '[va] "=&v"(va)',
             '[rn] "=&s"(nv)']
    ins = ['[addr] "v"(addr)', '[tp] "s"(next)'] + [f'[r{j}] "s"(r[{j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)] + ['"m0"', '"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out += prefetch_store(dw)
    out.append("}")
    return "\n".join(out)


THREAD_CONFIGS = [
    # threaded-jump flavour: name, DMs per wave, samples per lane, window, waves per SIMD
    ("t_f32_d8_k12_w48", 8, 12, 48, 3),
    ("t_f32_d8_k20_w56", 8, 20, 56, 2),
    ("t_f32_d4_k20_w56", 4, 20, 56, 3),
    ("t_f32_d4_k12_w48", 4, 12, 48, 4),
]

# fixed SGPRs of the threaded blocks: the block table's address and the jump target
TPC, TTG = 88, 90


def thread_layout(dw, k, wmax):
    """Byte layout of the threaded block table (shared with the host table
    builder through the generated constants): DW*NP plain blocks of PBS bytes,
    then DW*4 reload blocks of RBS bytes.

    plain block (j, o):  K v_add_f32_e32 (4 B each) reading window registers
                         o .. o+K-1, then the jump to DM j+1's block:
                         s_add_u32, s_addc_u32, s_setpc_b64 (4 B each); the
                         last DM's blocks end with s_branch to the exit and
                         two never-executed s_nop instead
    reload block (j, q): s_lshl_b32 + v_add_u32_e32 (LDS address of the
                         window start), WMAX/4 ds_read_b128 (8 B each),
                         s_waitcnt, then on DM 0 the scalar load of the next
                         channel's entries (8 B) or two s_nop elsewhere, then
                         K adds reading registers q .. q+K-1 and the jump."""
    np_ = wmax - k + 1
    pbs = 4 * k + 12
    rbs = 8 + 8 * (wmax // 4) + 4 + 8 + 4 * k + 12
    return np_, pbs, rbs


def gen_thread(name, dw, k, wmax, occ):
    """Threaded-jump flavour of the register-window step: no VGPR-relative
    addressing.  Each DM's table entry is the byte offset (within this step's
    block table) of a block of K plain adds whose window offset is fixed in
    the code; each block ends by jumping straight to the next DM's block, so a
    channel costs one computed jump per DM.  A DM whose run lies outside the
    current window takes a reload block, which loads the window at the DM's
    own start (entries DW..2DW-1 of the channel, in samples, a multiple of 4)
    and adds at sub-offset q = shift - start.  DM 0 always reloads.  The host
    builds and checks every entry (plan_jumptab); an offset outside the table
    would be a jump into arbitrary code, so the table is validated before it
    is uploaded."""
    assert k % 4 == 0 and wmax % 4 == 0 and wmax >= k + 4 and dw in (4, 8)
    wb = vgpr_budget(occ) - wmax
    np_, pbs, rbs = thread_layout(dw, k, wmax)
    nload = "s_load_dwordx8" if dw == 4 else "s_load_dwordx16"
    vec = "int8v" if dw == 4 else "int16v"
    out = []
    out.append(f"// {name}: DW={dw} K={k} WMAX={wmax} OCC={occ}, window v{wb}..v{wb + wmax - 1}, "
               f"{dw * np_} plain blocks of {pbs} B, {dw * 4} reload blocks of {rbs} B")
    up = name.upper()
    out.append(f"#define DD_{up}_NP {np_}")
    out.append(f"#define DD_{up}_PBS {pbs}")
    out.append(f"#define DD_{up}_RBS {rbs}")
    out.append(f"__device__ __forceinline__ void dd_{name}_channel(float* acc, const int* e, unsigned addr, const int32_t* next, int* en) {{")
    out += ["  unsigned va;", f"  {vec} nv;"]
    out.append("  asm volatile(")
    out.append(f'      "s_getpc_b64 s[{TPC}:{TPC + 1}]\\n"')
    out.append('      ".Lpc%=:\\n"')
    out.append(f'      "s_add_u32 s{TPC}, s{TPC}, .Ltab%=-.Lpc%=\\n"')
    out.append(f'      "s_addc_u32 s{TPC + 1}, s{TPC + 1}, 0\\n"')
    out.append(f'      "s_add_u32 s{TTG}, s{TPC}, %[o0]\\n"')
    out.append(f'      "s_addc_u32 s{TTG + 1}, s{TPC + 1}, 0\\n"')
    out.append(f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"')
    out.append('      ".p2align 6\\n"')
    out.append('      ".Ltab%=:\\n"')

    def tail(j):
        if j < dw - 1:
            return [f'      "s_add_u32 s{TTG}, s{TPC}, %[o{j + 1}]\\n"',
                    f'      "s_addc_u32 s{TTG + 1}, s{TPC + 1}, 0\\n"',
                    f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"']
        return ['      "s_branch .Lend%=\\n"', '      "s_nop 0\\n"', '      "s_nop 0\\n"']

    def adds(j, o):
        return [f'      "v_add_f32_e32 %[a{j}_{i}], v{wb + o + i}, %[a{j}_{i}]\\n"' for i in range(k)]

    def place(label, off):
        return [f'      "{label}:\\n"',
                f'      ".if ({label}-.Ltab%=) != {off}\\n .error \\"block table misplaced\\"\\n .endif\\n"']

    for j in range(dw):
        for o in range(np_):
            out += place(f".Lp%=_{j}_{o}", (j * np_ + o) * pbs)
            out += adds(j, o)
            out += tail(j)
    base = dw * np_ * pbs
    for j in range(dw):
        for q in range(4):
            out += place(f".Lr%=_{j}_{q}", base + (j * 4 + q) * rbs)
            out.append(f'      "s_lshl_b32 s{TTG}, %[s{j}], 2\\n"')
            out.append(f'      "v_add_u32_e32 %[va], s{TTG}, %[addr]\\n"')
            for i in range(wmax // 4):
                off = f" offset:{16 * i}" if i else ""
                out.append(f'      "ds_read_b128 v[{wb + 4 * i}:{wb + 4 * i + 3}], %[va]{off}\\n"')
            out.append('      "s_waitcnt lgkmcnt(0)\\n"')
            if j == 0:
                out.append(f'      "{nload} %[rn], %[tp], 0\\n"')
            else:
                out += ['      "s_nop 0\\n"', '      "s_nop 0\\n"']
            out += adds(j, q)
            out += tail(j)
    out.append('      ".Lend%=:\\n"')
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[va] "=&v"(va)', '[rn] "=&s"(nv)']
    ins = ['[addr] "v"(addr)', '[tp] "s"(next)']
    ins += [f'[o{j}] "s"(e[{j}])' for j in range(dw)]
    ins += [f'[s{j}] "s"(e[{dw + j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)]
    clob += [f'"s{i}"' for i in (TPC, TPC + 1, TTG, TTG + 1)] + ['"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out.append(f"  for (int i = 0; i < {2 * dw}; i++) en[i] = nv[i];")
    out.append("}")
    return "\n".join(out)


def shared_layout(dw, k):
    """Byte layout of the shared-window block table: DW*NP plain blocks of PBS
    bytes, then DW*4 reload blocks of RBS bytes (window of 4K floats, NP =
    3K+1 window offsets).  A lane loads the first 3K samples of its window
    from LDS; the last K are the next lane's samples 2K..3K-1 (lane l+1's
    window starts K samples after lane l's), read by DPP.

    plain block (j, o):  K adds (o+i < 3K: own registers, 4 B each;
                         3K <= o+i: DPP from the next lane, 8 B), then the jump
                         to DM j+1's block (12 B), padded with s_nop to the
                         largest block (8K + 12 B)
    reload block (j, q): v_lshl_add_u32 (8 B), 3K/4 ds_read_b128 (8 B each)
                         (DM 0's are issued before its block, so its block
                         starts at the next item), a partial s_waitcnt, K adds
                         of registers q..q+K-1 (4 B each), s_waitcnt for the
                         whole window, on DM 0 the scalar load of the next
                         channel's entries (8 B), and the jump; padded with
                         never-executed s_nop to the largest"""
    np_ = 3 * k + 1
    pbs = 8 * k + 12
    rbs = 8 + 8 * (3 * k // 4) + 4 + 8 + 4 * k + 12
    return np_, pbs, rbs


STAGE_CONFIGS = [
    # shared-window step that runs a whole stage of channels: name, DMs per
    # wave, samples per lane, waves per SIMD
    ("v_f32_d8_k12", 8, 12, 3),
    ("v_f32_d6_k12", 6, 12, 4),
    ("v_f32_d4_k12", 4, 12, 5),
]
# the stage step keeps a channel's entries in SGPRs it names itself: the
# current channel's 2*DW words from SA, the next channel's (scalar load
# target, 16 words) from SB
SA, SB = 56, 72


def gen_stage(name, dw, k, occ, fast=False):
    """Shared-window threaded-jump step that runs every channel of one stage.

    A lane owns K consecutive output samples of DW trial DMs; lane l's window
    of 4K staged samples starts K samples after lane l-1's.  For one channel
    each DM's table entry names the block that adds its K-sample run at its
    offset in the window (the offset is fixed in the block's code), and every
    block ends by jumping straight to the next DM's block.  A DM whose run
    lies outside the current window takes a reload block: it reads samples
    0..3K-1 of the window from LDS (3K/4 ds_read_b128) at the DM's own start;
    adds at window positions 3K..4K-1 read the next lane's positions 2K..3K-1
    through a DPP wave shift.  Only plain VGPR-operand adds pair up across
    the SIMD's two VALU pipes on gfx950 (DPP, SGPR-operand and three-source
    forms issue on one pipe at half rate), so the window is loaded rather
    than shifted into place, and DPP is left to the rare far offsets.

    A scalar instruction also costs issue time (about one per CU per clock),
    so the channel loop, the entry hand-over (DW s_mov_b64 from the scalar
    load target SB to the live set SA), the LDS address and the table offset
    advance are inside the assembly.

    In: acc, the first channel's entries as DW SGPR pairs (returned holding
    the entries of the channel after the stage), the first channel's LDS
    address, the LDS stride between channels, the wavefront's table base, the
    table's bytes per channel (the workgroup's DMs x 8), the byte offset of
    the next channel's entries (advanced per channel), and the channel count
    minus one.

    fast: each jump is s_add_u32 + s_setpc_b64 (the high word of the target
    is the table's, set once), which holds while no block offset carries out
    of the low 32 bits of the table address.  The step checks that on entry
    (the table's low word plus its size must not carry) and, if it would,
    returns 0 at once having changed nothing, so the caller runs the plain
    flavour; otherwise it returns 1."""
    assert k % 4 == 0 and 2 <= dw <= 8
    wb = vgpr_budget(occ) - 3 * k
    va = wb
    np_, pbs, rbs = shared_layout(dw, k)
    nload = "s_load_dwordx8" if 2 * dw <= 8 else "s_load_dwordx16"
    nb = 8 if 2 * dw <= 8 else 16
    out = []
    out.append(f"// {name}: DW={dw} K={k} OCC={occ}, window v{va}..v{va + 3 * k - 1}, "
               f"entries s{SA}.. (next: s{SB}..), "
               f"{dw * np_} plain blocks of {pbs} B, {dw * 4} reload blocks of {rbs} B")
    up = name.upper()
    out.append(f"#define DD_{up}_NP {np_}")
    out.append(f"#define DD_{up}_PBS {pbs}")
    out.append(f"#define DD_{up}_RBS {rbs}")
    out.append(f"#define DD_{up}_WMAX {4 * k}")
    table_bytes = dw * np_ * pbs + dw * 4 * rbs
    sfx = "stagef" if fast else "stage"
    ret = "int" if fast else "void"
    out.append(f"__device__ __forceinline__ {ret} dd_{name}_{sfx}(float* acc, int2v* e, unsigned addr, "
               f"unsigned lstride, const int32_t* tab, unsigned tstride, unsigned* toff, int cnt) {{")
    out.append("  unsigned va;")
    if fast:
        out.append("  int ok;")
    out.append("  asm volatile(")
    out.append(f'      "s_getpc_b64 s[{TPC}:{TPC + 1}]\\n"')
    out.append('      ".Lpc%=:\\n"')
    out.append(f'      "s_add_u32 s{TPC}, s{TPC}, .Ltab%=-.Lpc%=\\n"')
    out.append(f'      "s_addc_u32 s{TPC + 1}, s{TPC + 1}, 0\\n"')
    if fast:
        out.append('      "s_mov_b32 %[ok], 0\\n"')
        out.append(f'      "s_add_u32 s{TTG}, s{TPC}, {table_bytes}\\n"')
        out.append('      "s_cbranch_scc1 .Lout%=\\n"')
        out.append('      "s_mov_b32 %[ok], 1\\n"')
        out.append(f'      "s_mov_b32 s{TTG + 1}, s{TPC + 1}\\n"')
    for i in range(dw):
        out.append(f'      "s_mov_b64 s[{SA + 2 * i}:{SA + 2 * i + 1}], %[e{i}]\\n"')

    def window_load(start_reg):
        # DM 0's window (it always reloads), read ahead of its block: 3K/4
        # ds_read_b128 from the window start (samples) * 4 + the LDS address
        w = [f'      "v_lshl_add_u32 %[va], s{start_reg}, 2, %[addr]\\n"']
        for i in range(3 * k // 4):
            off = f" offset:{16 * i}" if i else ""
            w.append(f'      "ds_read_b128 v[{va + 4 * i}:{va + 4 * i + 3}], %[va]{off}\\n"')
        return w

    out += window_load(SA + dw)
    out.append('      ".Lchan%=:\\n"')
    out.append(f'      "s_add_u32 s{TTG}, s{TPC}, s{SA}\\n"')
    if not fast:
        out.append(f'      "s_addc_u32 s{TTG + 1}, s{TPC + 1}, 0\\n"')
    out.append(f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"')
    out.append('      ".p2align 6\\n"')
    out.append('      ".Ltab%=:\\n"')

    def tail(j):
        if j < dw - 1:
            if fast:  # same 12 bytes; the s_nop after the jump never runs
                return [f'      "s_add_u32 s{TTG}, s{TPC}, s{SA + j + 1}\\n"',
                        f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"',
                        '      "s_nop 0\\n"']
            return [f'      "s_add_u32 s{TTG}, s{TPC}, s{SA + j + 1}\\n"',
                    f'      "s_addc_u32 s{TTG + 1}, s{TPC + 1}, 0\\n"',
                    f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"']
        return ['      "s_branch .Lnext%=\\n"', '      "s_nop 0\\n"', '      "s_nop 0\\n"']

    def add(j, i, w):
        if w < 3 * k:
            return f'      "v_add_f32_e32 %[a{j}_{i}], v{va + w}, %[a{j}_{i}]\\n"', 4
        # the next lane's window position w - K (its window starts K later)
        return (f'      "v_add_f32_dpp %[a{j}_{i}], v{va + w - k}, %[a{j}_{i}] '
                f'wave_shl:1 row_mask:0xf bank_mask:0xf\\n"', 8)

    def place(label, off):
        return [f'      "{label}:\\n"',
                f'      ".if ({label}-.Ltab%=) != {off}\\n .error \\"block table misplaced\\"\\n .endif\\n"']

    for j in range(dw):
        for o in range(np_):
            out += place(f".Lp%=_{j}_{o}", (j * np_ + o) * pbs)
            size = 0
            for i in range(k):
                line, n = add(j, i, o + i)
                out.append(line)
                size += n
            out += tail(j)
            size += 12
            assert (pbs - size) % 4 == 0
            out += ['      "s_nop 0\\n"'] * ((pbs - size) // 4)
    base = dw * np_ * pbs
    for j in range(dw):
        for q in range(4):
            out += place(f".Lr%=_{j}_{q}", base + (j * 4 + q) * rbs)
            # The block's own adds read registers q..q+K-1 (q + i < K + 3 <=
            # 3K: own registers only), which the first K/4 + 1 of the 3K/4
            # window reads fill; LDS reads complete in order, so once at most
            # K/2 - 1 LDS/scalar operations are outstanding those have landed
            # (an older scalar load still in flight only means more have).
            # The rest of the window, which the later DMs' blocks read, is
            # waited for after the adds.
            early = f'      "s_waitcnt lgkmcnt({k // 2 - 1})\\n"'
            if j == 0:
                # the window was issued before the jump here (stage entry or
                # the previous channel's tail): wait for its first reads, add,
                # wait for the rest, then fetch the next channel's entries
                out.append(early)
                for i in range(k):
                    out.append(add(j, i, q + i)[0])
                out.append('      "s_waitcnt lgkmcnt(0)\\n"')
                out.append(f'      "{nload} s[{SB}:{SB + nb - 1}], %[tp], %[toff]\\n"')
                out += tail(j)
                used = 4 + 4 * k + 4 + 8 + 12
                assert (rbs - used) % 4 == 0 and used <= rbs
                out += ['      "s_nop 0\\n"'] * ((rbs - used) // 4)  # never executed
                continue
            # window start (samples) * 4 + the channel's LDS address: 8 B
            out.append(f'      "v_lshl_add_u32 %[va], s{SA + dw + j}, 2, %[addr]\\n"')
            for i in range(3 * k // 4):
                off = f" offset:{16 * i}" if i else ""
                out.append(f'      "ds_read_b128 v[{va + 4 * i}:{va + 4 * i + 3}], %[va]{off}\\n"')
            out.append(early)
            for i in range(k):
                out.append(add(j, i, q + i)[0])
            out.append('      "s_waitcnt lgkmcnt(0)\\n"')
            out += tail(j)
            used = 8 + 8 * (3 * k // 4) + 4 + 4 * k + 4 + 12
            assert (rbs - used) % 4 == 0 and used <= rbs
            out += ['      "s_nop 0\\n"'] * ((rbs - used) // 4)  # never executed
    out.append('      ".Lnext%=:\\n"')
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    out.append('      "v_add_u32_e32 %[addr], %[ls], %[addr]\\n"')
    out.append('      "s_add_u32 %[toff], %[toff], %[ts]\\n"')
    out.append('      "s_sub_u32 %[cnt], %[cnt], 1\\n"')
    out.append('      "s_cbranch_scc1 .Llast%=\\n"')
    # another channel: its DM 0 window goes out first, then the hand-over
    out += window_load(SB + dw)
    for i in range(dw):
        out.append(f'      "s_mov_b64 s[{SA + 2 * i}:{SA + 2 * i + 1}], s[{SB + 2 * i}:{SB + 2 * i + 1}]\\n"')
    out.append('      "s_branch .Lchan%=\\n"')
    out.append('      ".Llast%=:\\n"')
    for i in range(dw):
        out.append(f'      "s_mov_b64 %[e{i}], s[{SB + 2 * i}:{SB + 2 * i + 1}]\\n"')
    if fast:
        out.append('      ".Lout%=:\\n"')
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[va] "=&v"(va)', '[addr] "+v"(addr)', '[toff] "+s"(*toff)', '[cnt] "+s"(cnt)']
    if fast:
        outs.append('[ok] "=&s"(ok)')
    outs += [f'[e{i}] "+s"(e[{i}])' for i in range(dw)]
    ins = ['[tp] "s"(tab)', '[ls] "s"(lstride)', '[ts] "s"(tstride)']
    clob = [f'"v{wb + i}"' for i in range(3 * k)]
    clob += [f'"s{i}"' for i in range(SA, SA + 2 * dw)] + [f'"s{i}"' for i in range(SB, SB + nb)]
    clob += [f'"s{i}"' for i in (TPC, TPC + 1, TTG, TTG + 1)] + ['"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    if fast:
        out.append("  return ok;")
    out.append("}")
    return "\n".join(out)


LINKED_CONFIGS = [
    # linked shared-window flavour: name, DMs per wave, samples per lane, waves per SIMD
    ("l_f32_d6_k12", 6, 12, 4),
]


def linked_layout(dw, k):
    """Byte layout of the linked block table: DW*NP plain blocks of PBS bytes
    (as the shared-window flavour), then DW*8 reload blocks of RBS bytes
    (window sub-offset q in 0..3, times 'first visit of the step' or not),
    then the exit at END."""
    np_ = 3 * k + 1
    pbs = 8 * k + 12
    rbs = 8 + 8 * (k // 2) + 4 + 8 + 8 * k + 4 + 4 * k + 12
    end = dw * np_ * pbs + dw * 8 * rbs
    return np_, pbs, rbs, end


def gen_linked(name, dw, k, occ):
    """Linked flavour of the shared-window step: the DMs of a wavefront are
    visited in an order chosen by the host for each step (so DMs that read
    the same LDS row run back to back).  A step's entries are: the offset of
    the first block, then one 'next' offset per DM slot (the block that runs
    after that slot's block; the exit for the last one), then one window
    start per slot (LDS float offset from the workgroup's LDS base, used by
    reload blocks).  Every block ends with the jump to its slot's 'next'.
    The first block of a step is always a 'first visit' reload block, which
    issues the scalar load of the next step's entries once its window has
    arrived; other reload blocks do not.  Windows are shared between lanes
    by DPP (lane l+1's window starts K samples after lane l's; lanes 62 and
    63 only supply data).  The host builds
    and checks every entry (plan_linkedtab)."""
    assert k % 4 == 0 and 2 <= dw <= 7  # 1 + 2*DW entries fit one s_load_dwordx16
    wmax = 4 * k
    wb = vgpr_budget(occ) - 3 * k
    va, vb = wb, wb + 2 * k
    np_, pbs, rbs, end = linked_layout(dw, k)
    out = []
    out.append(f"// {name}: DW={dw} K={k} OCC={occ}, run A v{va}..v{va + 2 * k - 1}, "
               f"run B v{vb}..v{vb + k - 1}, {dw * np_} plain blocks of {pbs} B, "
               f"{dw * 8} reload blocks of {rbs} B, exit at {end}")
    up = name.upper()
    out.append(f"#define DD_{up}_NP {np_}")
    out.append(f"#define DD_{up}_PBS {pbs}")
    out.append(f"#define DD_{up}_RBS {rbs}")
    out.append(f"#define DD_{up}_END {end}")
    out.append(f"#define DD_{up}_WMAX {wmax}")
    out.append(f"__device__ __forceinline__ void dd_{name}_step(float* acc, const int* e, unsigned addr, const int32_t* next, int* en) {{")
    out += ["  unsigned va;", "  int16v nv;"]
    out.append("  asm volatile(")
    out.append(f'      "s_getpc_b64 s[{TPC}:{TPC + 1}]\\n"')
    out.append('      ".Lpc%=:\\n"')
    out.append(f'      "s_add_u32 s{TPC}, s{TPC}, .Ltab%=-.Lpc%=\\n"')
    out.append(f'      "s_addc_u32 s{TPC + 1}, s{TPC + 1}, 0\\n"')
    out.append(f'      "s_add_u32 s{TTG}, s{TPC}, %[st]\\n"')
    out.append(f'      "s_addc_u32 s{TTG + 1}, s{TPC + 1}, 0\\n"')
    out.append(f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"')
    out.append('      ".p2align 6\\n"')
    out.append('      ".Ltab%=:\\n"')

    def tail(j):
        return [f'      "s_add_u32 s{TTG}, s{TPC}, %[n{j}]\\n"',
                f'      "s_addc_u32 s{TTG + 1}, s{TPC + 1}, 0\\n"',
                f'      "s_setpc_b64 s[{TTG}:{TTG + 1}]\\n"']

    def add(j, i, w):
        if w < 2 * k:
            return f'      "v_add_f32_e32 %[a{j}_{i}], v{va + w}, %[a{j}_{i}]\\n"', 4
        if w < 3 * k:
            return f'      "v_add_f32_e32 %[a{j}_{i}], v{vb + w - 2 * k}, %[a{j}_{i}]\\n"', 4
        return (f'      "v_add_f32_dpp %[a{j}_{i}], v{vb + w - 3 * k}, %[a{j}_{i}] '
                f'wave_shl:1 row_mask:0xf bank_mask:0xf\\n"', 8)

    def place(label, off):
        return [f'      "{label}:\\n"',
                f'      ".if ({label}-.Ltab%=) != {off}\\n .error \\"block table misplaced\\"\\n .endif\\n"']

    for j in range(dw):
        for o in range(np_):
            out += place(f".Lp%=_{j}_{o}", (j * np_ + o) * pbs)
            size = 0
            for i in range(k):
                line, n = add(j, i, o + i)
                out.append(line)
                size += n
            out += tail(j)
            size += 12
            out += ['      "s_nop 0\\n"'] * ((pbs - size) // 4)
    base = dw * np_ * pbs
    for j in range(dw):
        for f in range(2):
            for q in range(4):
                out += place(f".Lr%=_{j}_{f}_{q}", base + ((j * 2 + f) * 4 + q) * rbs)
                out.append(f'      "s_lshl_b32 s{TTG}, %[s{j}], 2\\n"')
                out.append(f'      "v_add_u32_e32 %[va], s{TTG}, %[addr]\\n"')
                for i in range(k // 2):
                    off = f" offset:{16 * i}" if i else ""
                    out.append(f'      "ds_read_b128 v[{va + 4 * i}:{va + 4 * i + 3}], %[va]{off}\\n"')
                out.append('      "s_waitcnt lgkmcnt(0)\\n"')
                if f == 0:
                    out.append('      "s_load_dwordx16 %[rn], %[tp], 0\\n"')
                else:
                    out += ['      "s_nop 0\\n"', '      "s_nop 0\\n"']
                for m in range(k):
                    out.append(f'      "v_mov_b32_dpp v{vb + m}, v{va + k + m} wave_shl:1 '
                               f'row_mask:0xf bank_mask:0xf\\n"')
                out.append('      "s_nop 1\\n"')
                for i in range(k):
                    out.append(add(j, i, q + i)[0])
                out += tail(j)
    out += place(".Lend%=", end)
    out.append('      "s_waitcnt lgkmcnt(0)\\n"')
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[va] "=&v"(va)', '[rn] "=&s"(nv)']
    ins = ['[addr] "v"(addr)', '[tp] "s"(next)', '[st] "s"(e[0])']
    ins += [f'[n{j}] "s"(e[{1 + j}])' for j in range(dw)]
    ins += [f'[s{j}] "s"(e[{1 + dw + j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(3 * k)]
    clob += [f'"s{i}"' for i in (TPC, TPC + 1, TTG, TTG + 1)] + ['"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out.append("  for (int i = 0; i < 16; i++) en[i] = nv[i];")
    out.append("}")
    return "\n".join(out)


def main():
    print("// Generated by gen_window_asm.py; do not edit by hand.")
    print("#pragma once")
    print("typedef int int2v __attribute__((ext_vector_type(2)));")
    print("typedef int int4v __attribute__((ext_vector_type(4)));")
    print("typedef int int8v __attribute__((ext_vector_type(8)));")
    print("typedef int int16v __attribute__((ext_vector_type(16)));")
    for cfg in CONFIGS:
        print(gen(*cfg))
        print()
    for cfg in CONFIGS:
        print(gen_sched(*cfg))
        print()
    for cfg in JT_CONFIGS:
        print(gen_jt(*cfg))
        print()
    for cfg in PAIR_CONFIGS:
        print(gen_pairs(*cfg))
        print()
    for cfg in THREAD_CONFIGS:
        print(gen_thread(*cfg))
        print()
    for cfg in LINKED_CONFIGS:
        print(gen_linked(*cfg))
        print()
    for cfg in STAGE_CONFIGS:
        print(gen_stage(*cfg))
        print()
        print(gen_stage(*cfg, fast=True))
        print()


if __name__ == "__main__":
    sys.exit(main())
