"""Per-kernel summary of rocprofv3 runs of `bench.py --profile-evals K`.

The profiled run launches a marker kernel (torch's spin kernel), K library
evaluations with the library's timing spans on, and a second marker, and
writes the span names in launch order (--profile-out). This script takes the
dispatches between the two markers from each rocprofv3 CSV, splits them into
the K evaluations, names them after the spans (each span owns the dispatches
from its first kernel up to the next span's first kernel) and averages:

  --trace      kernel-trace CSV (rocprofv3 --kernel-trace --output-format csv)
               -> average duration per launch
  --fetch/--write  FETCH_SIZE / WRITE_SIZE counter CSVs (KiB per dispatch),
               scaled by --copy-fetch/--copy-write, the same counters read for a
               plain device copy of --copy-bytes bytes (bench.py --copy-calib)
               -> HBM bytes per launch and per evaluation
  --sq         counter CSVs with SQ_* and GRBM_GUI_ACTIVE -> matrix-core busy,
               vector-ALU busy, issue-wait fraction, LDS bank conflicts

and writes a JSON record (read by bench.py while the library sources are
unchanged) and a Markdown table.

    python -m paper_2303_08169_amd.profile_summary --spans S.json --trace T.csv \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \
        --copy-bytes 1073741824 --sq Q.csv --agent A.csv --json out.json --md out.md
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import re
import sys

# First kernel of each timing span (by the kernel's own name); a span owns the
# dispatches from that kernel up to the first kernel of the next span.
SPAN_KERNELS = [
    (r"^neighbor_check_rebuild$", ("k_displacement",)),
    (r"^edge_list$", ("k_edge_count",)),
    (r"^chunk_view$", ("k_chunk_edges",)),
    (r"^geometry$", ("k_geometry",)),
    (r"^fwd\.twobody$", ("k_tb_fwd",)),
    (r"^bwd\.twobody$", ("k_tb_bwd",)),
    (r"^(fwd|bwd)\.", ("k_gemm", "k_gemm_ws")),
    (r"^tp_fwd\d+$", ("k_tp_fwd", "k_tp_fwd_last32")),
    (r"^tp_bwd\d+$", ("k_tp_bwd", "k_tp_bwd_last32")),
    (r"^env_fwd\d+$", ("k_env_fwd",)),
    (r"^env_bwd\d+$", ("k_env_adjoint",)),
    (r"^edge_energy$", ("k_edge_energy",)),
    (r"^atom_energy$", ("k_atom_energy",)),
    (r"^fill$", ("k_fill",)),
    (r"^geometry_bwd$", ("k_geometry_bwd",)),
    (r"^total_energy$", ("k_total_energy",)),
    (r"^forces$", ("k_forces",)),
    (r"^fused$", ("k_fused",)),
]
MARKER = "spin_kernel"


def base_name(kernel):
    """Library kernel's identifier (k_...) from a demangled rocprof name."""
    m = re.search(r"\b(k_[A-Za-z0-9_]+)", kernel)
    return m.group(1) if m else kernel


def span_kernels(span):
    for pat, names in SPAN_KERNELS:
        if re.search(pat, span):
            return names
    raise ValueError(f"no kernel known for span {span!r}")


def read_dispatches(path):
    """[(name, {counter: value}, duration_ns or None)] in dispatch order."""
    rows = list(csv.DictReader(open(path)))
    if not rows:
        return []
    if "Counter_Name" in rows[0]:
        by = collections.OrderedDict()
        for r in rows:
            d = by.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], collections.defaultdict(float), None])
            d[1][r["Counter_Name"]] += float(r["Counter_Value"])
        return [tuple(by[k]) for k in sorted(by)]
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    rows.sort(key=lambda r: (int(r["Start_Timestamp"]), int(r[key])))
    return [(r["Kernel_Name"], {}, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in rows]


def evaluations(disp, spans, evals):
    """Dispatches between the last two markers, split into `evals` groups that
    each start with the first span's kernel."""
    marks = [i for i, d in enumerate(disp) if MARKER in d[0]]
    if len(marks) < 2:
        raise ValueError("fewer than two marker dispatches")
    inner = disp[marks[-2] + 1: marks[-1]]
    first = span_kernels(spans[0])
    starts = [i for i, d in enumerate(inner) if base_name(d[0]) in first]
    if len(starts) != evals:
        raise ValueError(f"found {len(starts)} evaluations between the markers, expected {evals}")
    groups = [inner[a:b] for a, b in zip(starts, starts[1:] + [len(inner)])]
    if len(groups) > 1:
        # the last evaluation is followed by whatever ran before the marker
        # (a flag read-back): keep as many dispatches as the others have
        groups[-1] = groups[-1][:len(groups[0])]
    seq = [base_name(d[0]) for d in groups[0]]
    for g in groups[1:]:
        if [base_name(d[0]) for d in g] != seq:
            raise ValueError("evaluations launch different kernel sequences")
    return groups


def align(group, spans):
    """Index range [a, b) of the dispatches of every span in one evaluation."""
    starts, cur = [], 0
    for s in spans:
        names = span_kernels(s)
        while cur < len(group) and base_name(group[cur][0]) not in names:
            cur += 1
        if cur == len(group):
            raise ValueError(f"span {s!r}: none of {names} launched after the previous span")
        starts.append(cur)
        cur += 1
    return list(zip(starts, starts[1:] + [len(group)]))


def per_span(path, spans, evals):
    """{span: (kernel names, {counter: value per evaluation}, ns per evaluation)}."""
    groups = evaluations(read_dispatches(path), spans, evals)
    ranges = align(groups[0], spans)
    out = {}
    for s, (a, b) in zip(spans, ranges):
        tot = collections.defaultdict(float)
        ns = 0.0
        for g in groups:
            for name, ctr, dur in g[a:b]:
                for k, v in ctr.items():
                    tot[k] += v / evals
                if dur is not None:
                    ns += dur / evals
        out[s] = (sorted({base_name(d[0]) for d in groups[0][a:b]}), dict(tot), ns,
                  [d[0] for d in groups[0][a:b]])
    total = collections.defaultdict(float)
    for g in groups:
        for _, ctr, _ in g:
            for k, v in ctr.items():
                total[k] += v / evals
    return out, dict(total)


def per_kernel(path, spans, evals):
    """Like per_span, keyed by the library kernel's name (for evaluations that
    run some spans several times, e.g. in centre chunks): (kernel, counters
    per evaluation, ns per evaluation, launches per evaluation)."""
    groups = evaluations(read_dispatches(path), spans, evals)
    out = {}
    for g in groups:
        for name, ctr, dur in g:
            b = base_name(name)
            names, tot, ns, cnt = out.setdefault(b, ([b], collections.defaultdict(float), [0.0], [0]))
            for k, v in ctr.items():
                tot[k] += v / evals
            if dur is not None:
                ns[0] += dur / evals
            cnt[0] += 1
    res = {b: (names, dict(tot), ns[0], cnt[0] / evals) for b, (names, tot, ns, cnt) in out.items()}
    total = collections.defaultdict(float)
    for _, tot, _, _ in res.values():
        for k, v in tot.items():
            total[k] += v
    return res, dict(total)


def copy_scale(path, counter, nbytes):
    """nbytes / (KiB the counter reads for the largest plain device copy)."""
    best = 0.0
    for name, ctr, _ in read_dispatches(path):
        if "copyBuffer" in name and counter in ctr:
            best = max(best, ctr[counter])
    if best <= 0:
        raise ValueError(f"no copy dispatch with {counter} in {path}")
    return nbytes / (best * 1024.0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--spans", required=True)
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--sq", nargs="*", default=[])
    ap.add_argument("--agent", help="run_agent_info.csv of a counter run (SIMD, CU and XCC counts)")
    ap.add_argument("--stats", help="kernel-stats CSV of the trace run (rocprofv3 --stats): whole-run table")
    ap.add_argument("--commands", default="", help="text file with the commands that made the inputs")
    ap.add_argument("--json", required=True)
    ap.add_argument("--md", required=True)
    a = ap.parse_args(argv)

    prof = json.load(open(a.spans))
    spans, evals = prof["spans"], prof["evals"]
    # spans that run once per evaluation are named after the spans; otherwise
    # (centre chunks) the figures are per kernel
    by_span = all(c == evals for c in prof["span_counts"])

    def collect(path):
        if by_span:
            res, tot = per_span(path, spans, evals)
            return {k: (v[0], v[1], v[2], 1.0) for k, v in res.items()}, tot
        return per_kernel(path, spans, evals)

    rec = {"workload": prof["workload"], "precision": prof["precision"], "path": prof["path"],
           "edges": prof["edges"], "evals": evals, "source_sha256": prof["source_sha256"],
           "keyed_by": "span" if by_span else "kernel"}
    rows = collections.OrderedDict((s, {"kernels": None}) for s in spans) if by_span else collections.OrderedDict()
    if a.trace:
        ts, _ = collect(a.trace)
        for s, (names, _, ns, per) in ts.items():
            rows.setdefault(s, {}).update(kernels=names, avg_ms_trace=ns * 1e-6 / per, launches_per_eval=per,
                                          ms_per_eval=ns * 1e-6)
    if a.fetch and a.write:
        fs = copy_scale(a.copy_fetch, "FETCH_SIZE", a.copy_bytes)
        ws = copy_scale(a.copy_write, "WRITE_SIZE", a.copy_bytes)
        rec.update(fetch_scale=fs, write_scale=ws)
        f, ftot = collect(a.fetch)
        w, wtot = collect(a.write)
        for s in f:
            fk, wk = f[s][1].get("FETCH_SIZE", 0.0), w.get(s, f[s])[1].get("WRITE_SIZE", 0.0)
            per = f[s][3]
            rows.setdefault(s, {}).update(fetch_kib=fk / per, write_kib=wk / per,
                                          hbm_bytes_per_launch=1024.0 * (fk * fs + wk * ws) / per,
                                          kernels=rows.get(s, {}).get("kernels") or f[s][0])
        rec["hbm_bytes_per_step"] = 1024.0 * (ftot.get("FETCH_SIZE", 0.0) * fs + wtot.get("WRITE_SIZE", 0.0) * ws)
    agent = {}
    if a.agent:
        for r in csv.DictReader(open(a.agent)):
            if r.get("Name", "").startswith("gfx"):
                agent = {k: int(r[k]) for k in ("Simd_Count", "Cu_Count", "Num_Xcc")}
        rec["agent"] = agent
    for path in a.sq:
        q, _ = collect(path)
        for s in q:
            rows.setdefault(s, {}).setdefault("sq", {}).update(q[s][1])
    for s in rows:
        c = rows[s].get("sq")
        if not c or "GRBM_GUI_ACTIVE" not in c or not agent:
            continue
        cyc = c["GRBM_GUI_ACTIVE"] / agent["Num_Xcc"]  # the counter is summed over the XCDs
        d = {}
        if "SQ_VALU_MFMA_BUSY_CYCLES" in c:
            d["mfma_busy"] = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (agent["Simd_Count"] * cyc)
        if "SQ_ACTIVE_INST_VALU" in c:
            d["valu_busy"] = c["SQ_ACTIVE_INST_VALU"] / (agent["Cu_Count"] * cyc)
        if "SQ_WAIT_INST_ANY" in c and "SQ_WAVE_CYCLES" in c:
            d["wait_any"] = c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"]
        if "SQ_LDS_BANK_CONFLICT" in c and c.get("SQ_INSTS_LDS"):
            d["lds_bank_conflict_per_lds_inst"] = c["SQ_LDS_BANK_CONFLICT"] / c["SQ_INSTS_LDS"]
        if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in c:
            d["mfma_bf16_flop_counted"] = 512.0 * c["SQ_INSTS_VALU_MFMA_MOPS_BF16"]
        if rows[s].get("ms_per_eval"):
            d["clock_ghz_implied"] = cyc / (rows[s]["ms_per_eval"] * 1e6)
        rows[s].update(d)
    for r in rows.values():
        r.pop("sq", None)  # raw counter sums: only the fractions above are kept
    rec["spans" if by_span else "kernels"] = rows
    rec["source_file"] = a.md.split("/")[-1]
    with open(a.json, "w") as fh:
        json.dump(rec, fh, indent=1)

    cmds = open(a.commands).read().strip() if a.commands else ""
    out = [f"# Per-kernel profile: {prof['workload']}, {prof['precision']}, {prof['path']} path",
           "", f"{evals} evaluations of {prof['edges']:,} edges between two marker kernels "
           "(`bench.py --profile-evals`), averaged per evaluation.", ""]
    if cmds:
        out += ["Commands (R: the repository root on the machine that ran them; one counter set per run):", "", "```", cmds, "```", ""]
    if "fetch_scale" in rec:
        out += [f"HBM bytes = 1024 x (FETCH_SIZE x {rec['fetch_scale']:.4f} + WRITE_SIZE x {rec['write_scale']:.4f}); "
                f"the factors make a plain device copy of {a.copy_bytes / 2**20:,.0f} MiB read and write exactly that "
                "many bytes.", "",
                f"HBM bytes per evaluation (all kernels): {rec['hbm_bytes_per_step'] / 1e9:.2f} GB.", ""]
    if not by_span:
        out += ["Centre chunks run some spans several times per evaluation, so the rows are the library's "
                "kernels (all their launches in one evaluation).", ""]
    hdr = ["span" if by_span else "kernel", "kernels", "launches", "avg ms (trace)", "HBM GB/launch", "MFMA busy", "VALU busy", "issue wait",
           "LDS conflicts/inst", "clock GHz"]
    out += ["| " + " | ".join(hdr) + " |", "|" + "---|" * len(hdr)]

    def f_(v, fmt):
        return "-" if v is None else format(v, fmt)

    for s in sorted(rows, key=lambda s: -(rows[s].get("ms_per_eval") or 0)):
        r = rows[s]
        hb = r.get("hbm_bytes_per_launch")
        out.append("| " + " | ".join([
            s, ", ".join(r.get("kernels") or []), f_(r.get("launches_per_eval"), ".0f"),
            f_(r.get("avg_ms_trace"), ".3f"),
            f_(hb / 1e9 if hb is not None else None, ".3f"), f_(r.get("mfma_busy"), ".3f"),
            f_(r.get("valu_busy"), ".3f"), f_(r.get("wait_any"), ".3f"),
            f_(r.get("lds_bank_conflict_per_lds_inst"), ".3f"), f_(r.get("clock_ghz_implied"), ".2f")]) + " |")
    if a.stats:
        st = list(csv.DictReader(open(a.stats)))
        st.sort(key=lambda r: -float(r["TotalDurationNs"]))
        out += ["", "Whole profiled run (rocprofv3 --stats; includes the two warm-up calls, so 7 calls of each "
                "kernel of an evaluation):", "", "| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
        for r in st[:20]:
            out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.3f} | "
                       f"{float(r['AverageNs']) * 1e-6:.3f} | {float(r['Percentage']):.2f} |")
    out += ["", f"Library sources SHA-256: `{prof['source_sha256']}` (bench.py uses these figures only while the "
            "sources hash to this value)."]
    with open(a.md, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(f"wrote {a.json} and {a.md}", file=sys.stderr)


if __name__ == "__main__":
    main()
