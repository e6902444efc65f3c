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
    out.append(f"__device__ __forceinline__ void dd_{name}_channel(float* acc, const int* r, unsigned addr) {{")
    out.append("  int ws, ix, tb;")
    out.append("  unsigned va;")
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
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[ws] "=&s"(ws)', '[ix] "=&s"(ix)', '[tb] "=&s"(tb)', '[va] "=&v"(va)']
    ins = ['[addr] "v"(addr)'] + [f'[r{j}] "s"(r[{j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)] + ['"m0"', '"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
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
    out.append(f"__device__ __forceinline__ void dd_{name}_channel(float* acc, const int* r, unsigned addr) {{")
    out.append("  int ws, ix, tb;")
    out.append("  unsigned va;")
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
    outs = []
    for j in range(dw):
        for kk in range(k):
            outs.append(f'[a{j}_{kk}] "+v"(acc[{j * k + kk}])')
    outs += ['[ws] "=&s"(ws)', '[ix] "=&s"(ix)', '[tb] "=&s"(tb)', '[va] "=&v"(va)']
    ins = ['[addr] "v"(addr)'] + [f'[r{j}] "s"(r[{j}])' for j in range(dw)]
    clob = [f'"v{wb + i}"' for i in range(wmax)] + [f'"s{i}"' for i in (PC_LO, PC_HI, T_LO, T_HI)]
    clob += ['"scc"', '"memory"']
    out.append("      : " + ",\n        ".join(outs))
    out.append("      : " + ", ".join(ins))
    out.append("      : " + ", ".join(clob) + ");")
    out.append("}")
    return "\n".join(out)


def main():
    print("// Generated by gen_window_asm.py; do not edit by hand.")
    print("#pragma once")
    for cfg in CONFIGS:
        print(gen(*cfg))
        print()
    for cfg in JT_CONFIGS:
        print(gen_jt(*cfg))
        print()


if __name__ == "__main__":
    sys.exit(main())
