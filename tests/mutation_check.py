"""Mutation check of the oracle's pins (CPU only, test infrastructure).

Plants one plausible mistake at a time (a wrong constant, sign, index,
rounding rule, tie rule, normalisation, FFT direction, ...) in a scratch copy
of the oracle, rebuilds the copy's C library when the C source changed, and
runs the copy's CPU test suite, which must fail for every mistake.  The first
entry plants nothing and must pass.

    python tests/mutation_check.py [name prefix ...]

The scratch copy is made in .mutation_scratch at the repository root and
removed at the end.
"""
import os, shutil, subprocess, sys
R = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
M = os.path.join(R, ".mutation_scratch")
C = "oracle/dd_oracle.c"
P = "oracle/__init__.py"
MUTS = [
    ("B0 baseline (no mutation)", P, "def max_shift(", "def max_shift("),
    ("C1 constant 4150->4148", C, "4150.0 *", "4148.0 *"),
    ("C2 delay sign", C, "(1.0 / (f_c * f_c) - 1.0 / (f_top * f_top))", "(1.0 / (f_top * f_top) - 1.0 / (f_c * f_c))"),
    ("C3 channel freq off by one", C, "return f_top - (double)c * df;", "return f_top - (double)(c + 1) * df;"),
    ("C4 rounding floor", C, "(int64_t)llround(x)", "(int64_t)floor(x)"),
    ("C5 dropped last channel", C, "      for (int64_t c = 0; c < nchans; c++) {", "      for (int64_t c = 0; c < nchans - 1; c++) {"),
    ("C6 reversed delay index", C, "in + c * stride + t_begin + dl[c]", "in + c * stride + t_begin + dl[nchans - 1 - c]"),
    ("C7 f16 subnormal exponent", C, "ldexp((double)m, -24)", "ldexp((double)m, -25)"),
    ("C8 f16 normal exponent", C, "ldexp((double)(1024 + m), e - 25)", "ldexp((double)(1024 + m), e - 24)"),
    ("P1 detect sample std", P, "sigma = r.std()", "sigma = r.std(ddof=1)"),
    ("P2 detect tie to widest", P, "better = s > best[: nout - w + 1]", "better = s >= best[: nout - w + 1]"),
    ("P3 detect sqrt(w) dropped", P, "/ (sigma * np.sqrt(w))", "/ (sigma * w)"),
    ("P4 corner flip wrong axis", P, "x = x[:, ::-1]", "x = x[::-1, :]"),
    ("P5 bin sum not mean", P, "sum(axis=2) / b", "sum(axis=2)"),
    ("P6 channel bin off by one", P, "(nfft // 2 - 1 - j) % nfft", "(nfft // 2 - j) % nfft"),
    ("P7 inverse FFT", P, "X = np.fft.fft(blocks, axis=1)", "X = np.fft.ifft(blocks, axis=1) * nfft"),
    ("P8 max_shift + 1", P, "return int(np.max(delays))", "return int(np.max(delays)) + 1"),
    ("P9 one fine DM fewer", P, "nfine = int(math.ceil((dm_hi - dm_lo) / ddm - 1e-9))", "nfine = int(math.ceil((dm_hi - dm_lo) / ddm - 1e-9)) - 1"),
    ("P10 delay rounding half-even", C, "(int64_t)llround(x)", "(int64_t)nearbyint(x)"),
    ("C9 t_begin ignored", C, "in + c * stride + t_begin + dl[c]", "in + c * stride + dl[c]"),
    ("C10 u8 read as signed", C, "#define CONV_U8(x) ((int64_t)(x))", "#define CONV_U8(x) ((int64_t)(int8_t)(x))"),
    ("C11 f32 summed in float", C, "DEFINE_DEDISP(orc_dedisperse_f32, float, double, CONV_F32)",
     "DEFINE_DEDISP(orc_dedisperse_f32_unused, float, double, CONV_F32)\n"
     "static int orc_f32_float_acc(const float* in, int64_t nchans, int64_t nsamp, int64_t stride, const int64_t* delays,"
     " int32_t ndms, const int32_t* rows, int32_t nrows, int64_t t_begin, int64_t t_end, double* out, int32_t nthreads) {"
     " int rc = orc_dedisperse_f32_unused(in, nchans, nsamp, stride, delays, ndms, rows, nrows, t_begin, t_end, out, nthreads);"
     " if (rc != ORC_OK) return rc; int64_t n = t_end - t_begin;"
     " for (int32_t i = 0; i < nrows; i++) { const int64_t* dl = delays + (int64_t)rows[i] * nchans;"
     " for (int64_t t = 0; t < n; t++) { float a = 0.f; for (int64_t c = 0; c < nchans; c++) a += in[c * stride + t_begin + t + dl[c]];"
     " out[(int64_t)i * n + t] = a; } } return ORC_OK; }\n"
     "int orc_dedisperse_f32(const float* in, int64_t nchans, int64_t nsamp, int64_t stride, const int64_t* delays,"
     " int32_t ndms, const int32_t* rows, int32_t nrows, int64_t t_begin, int64_t t_end, double* out, int32_t nthreads) {"
     " return orc_f32_float_acc(in, nchans, nsamp, stride, delays, ndms, rows, nrows, t_begin, t_end, out, nthreads); }"),
    ("P13 nominal DM at range start", P, "nominal = dm_lo + (np.arange(nnom, dtype=np.float64) + 0.5) * dsub",
     "nominal = dm_lo + np.arange(nnom, dtype=np.float64) * dsub"),
    ("P14 subband top off by one", P, "t1 = dn[:, c0:c0 + cps] - dn[:, [c0]]", "t1 = dn[:, c0:c0 + cps] - dn[:, [min(c0 + 1, nchans - 1)]] + 1"),
    ("P15 stage 2 at bottom channel", P, "df_tab = delay_table(nchans, f_top, df, ts, fine)[:, tops]",
     "df_tab = delay_table(nchans, f_top, df, ts, fine)[:, np.minimum(tops + cps - 1, nchans - 1)]"),
    ("P16 nominal index rounded", P, "np.floor((fine - dm_lo) / dsub)", "np.round((fine - dm_lo) / dsub)"),
    ("P17 binning ignored in delays", P, "        ts = t_samp * b\n", "        ts = t_samp\n"),
    ("P11 threshold strict", P, "t = np.nonzero(best >= nsigma)[0]", "t = np.nonzero(best > nsigma)[0]"),
    ("P12 corner flip ignored", P, "    if flip:\n        x = x[:, ::-1]", "    if False:\n        x = x[:, ::-1]"),
]
only = sys.argv[1:]
res = []
for name, f, old, new in MUTS:
    if only and not any(name.startswith(o) for o in only):
        continue
    if os.path.exists(M):
        shutil.rmtree(M)
    os.makedirs(M)
    for d in ("oracle", "synth", "tests", "paper_1107_2516_amd", "include"):
        shutil.copytree(os.path.join(R, d), os.path.join(M, d),
                        ignore=shutil.ignore_patterns("__pycache__", "_build", "*.tmp"))
    for extra in ("__graft_entry__.py", "pytest.ini", "conftest.py", "setup.cfg", "pyproject.toml"):
        if os.path.exists(os.path.join(R, extra)):
            shutil.copy(os.path.join(R, extra), M)
    path = os.path.join(M, f)
    s = open(path).read()
    assert s.count(old) == 1, (name, s.count(old))
    open(path, "w").write(s.replace(old, new))
    if f.endswith(".c"):
        subprocess.run([sys.executable, "-m", "oracle.build"], cwd=M, check=True, capture_output=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-m", "not gpu", "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=M, capture_output=True, text=True, timeout=600)
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED") or l.startswith("ERROR")]
    planted = old != new
    ok = (r.returncode != 0) == planted
    res.append((name, planted, ok))
    verdict = ("caught" if r.returncode else "MISSED") if planted else ("passes" if ok else "FAILS")
    print(f"{name:32s} {verdict} {failed[:1]}", flush=True)
shutil.rmtree(M, ignore_errors=True)
n = sum(1 for _, p, _ in res if p)
print(f"caught {sum(1 for _, p, ok in res if p and ok)} of {n} planted mistakes; "
      f"unmutated copy {'passes' if all(ok for _, p, ok in res if not p) else 'FAILS'}")
sys.exit(0 if all(ok for _, _, ok in res) else 1)
