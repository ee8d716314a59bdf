"""Library-call substitution in C host programs (the paper's section 3.4,
steps A-1, B-1, C-1 and the interface check of C-2).

* A-1: the source is scanned for calls of external library functions listed
  in the code pattern table (`patterns.json`): an identifier followed by an
  argument list, outside comments, string and character literals, that the
  file does not define itself.
* B-1: each detected name is looked up in the table; its record gives the
  replacement of the same meaning in libfb and the usage method that connects
  it (an adapter function with the library function's signature).
* C-2: the call's argument count must equal the recorded signature's; a call
  that does not match is reported and left as it is (the paper asks the user
  instead of changing the interface).
* C-1: matching calls are renamed to the adapter, the replacement's header is
  included and the adapter is inserted after the includes.  The rewritten
  program links libfb instead of the CPU library.

Usage:  python -m paper_2004_09883_amd.substitute app.c -o app_fb.c
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys

PATTERNS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "patterns.json")

_IDENT = re.compile(r"[A-Za-z_][A-Za-z0-9_]*")


def load_patterns(path: str = PATTERNS) -> dict:
    """Function name -> record (with the owning library's name and header)."""
    with open(path) as f:
        db = json.load(f)
    table = {}
    for lib in db["libraries"]:
        for name, rec in lib["functions"].items():
            table[name] = dict(rec, library=lib["library"], library_header=lib["header"])
    return table


def blank_comments_and_literals(src: str) -> str:
    """The source with comments, string and character literals replaced by
    spaces (newlines kept), so that offsets and line numbers still match."""
    out = list(src)
    i, n = 0, len(src)

    def blank(a, b):
        for k in range(a, b):
            if out[k] != "\n":
                out[k] = " "

    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            j = n if j < 0 else j
            blank(i, j)
            i = j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            j = n if j < 0 else j + 2
            blank(i, j)
            i = j
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            j = min(n, j + 1)
            blank(i + 1, j - 1)
            i = j
        else:
            i += 1
    return "".join(out)


def _args(code: str, open_paren: int):
    """Argument texts of the call whose '(' is at open_paren, and the offset
    after its ')'; None when the parentheses do not balance."""
    depth, start, args = 0, open_paren + 1, []
    for k in range(open_paren, len(code)):
        ch = code[k]
        if ch in "([{":
            depth += 1
        elif ch in ")]}":
            depth -= 1
            if depth == 0:
                last = code[start:k].strip()
                if last or args:
                    args.append(last)
                return args, k + 1
        elif ch == "," and depth == 1:
            args.append(code[start:k].strip())
            start = k + 1
    return None


def _defined_here(code: str, name: str) -> bool:
    """True when the file defines `name` (a parameter list followed by a body)."""
    for m in re.finditer(r"\b%s\s*\(" % re.escape(name), code):
        r = _args(code, m.end() - 1)
        if r is None:
            continue
        rest = code[r[1]:].lstrip()
        if rest.startswith("{"):
            return True
    return False


def detect(src: str, table: dict):
    """A-1 and B-1: every call of a table function in `src`, as dicts with
    name, line, column, offset, argument texts, the record and whether the
    interface matches (C-2)."""
    code = blank_comments_and_literals(src)
    found = []
    for name in table:
        if _defined_here(code, name):
            continue
        for m in re.finditer(r"\b%s\s*\(" % re.escape(name), code):
            # a call, not a declaration: the previous token is not a type or identifier
            before = code[:m.start()].rstrip()
            prev = _IDENT.findall(before[-64:])
            if before and (before[-1].isalnum() or before[-1] == "_") and prev and prev[-1] not in ("return",):
                continue
            r = _args(code, m.end() - 1)
            if r is None:
                continue
            args = [src_slice.strip() for src_slice in _arg_source(src, m.end() - 1, r[1])]
            rec = table[name]
            line = code.count("\n", 0, m.start()) + 1
            col = m.start() - (code.rfind("\n", 0, m.start()) + 1) + 1
            found.append({"name": name, "line": line, "column": col, "offset": m.start(), "args": args,
                          "library": rec["library"], "replacement": rec["replacement"]["library"],
                          "adapter": rec["replacement"]["adapter"],
                          "interface_ok": len(args) == len(rec["params"]),
                          "expected_args": len(rec["params"])})
    found.sort(key=lambda d: d["offset"])
    return found


def _arg_source(src: str, open_paren: int, end: int):
    """The argument texts from the original source (literals intact)."""
    code = blank_comments_and_literals(src)
    depth, start, parts = 0, open_paren + 1, []
    for k in range(open_paren, end):
        ch = code[k]
        if ch in "([{":
            depth += 1
        elif ch in ")]}":
            depth -= 1
            if depth == 0:
                if src[start:k].strip() or parts:
                    parts.append(src[start:k])
                break
        elif ch == "," and depth == 1:
            parts.append(src[start:k])
            start = k + 1
    return parts


def rewrite(src: str, table: dict):
    """C-1: the rewritten source and the report of every detected call.
    Calls whose interface does not match are left unchanged (reported with
    "action": "ask the user")."""
    calls = detect(src, table)
    out = src
    used = {}
    for c in reversed(calls):   # from the end, so that earlier offsets stay valid
        if not c["interface_ok"]:
            c["action"] = "left unchanged: %d arguments, the library function takes %d; ask the user" % (
                len(c["args"]), c["expected_args"])
            continue
        out = out[:c["offset"]] + c["adapter"] + out[c["offset"] + len(c["name"]):]
        c["action"] = "replaced by %s (%s)" % (c["adapter"], c["replacement"])
        used[c["name"]] = table[c["name"]]
    if used:
        headers = sorted({rec["replacement"]["header"] for rec in used.values()})
        adapters = []
        for name in sorted(used):
            adapters.extend(used[name]["replacement"]["usage"])
        block = "".join('#include "%s"\n' % h for h in headers) + "\n" + "\n".join(adapters) + "\n"
        out = _insert_after_includes(out, block)
    return out, calls


def _insert_after_includes(src: str, block: str) -> str:
    lines = src.splitlines(keepends=True)
    last = -1
    for i, ln in enumerate(lines):
        if ln.lstrip().startswith("#include"):
            last = i
    pos = sum(len(ln) for ln in lines[:last + 1])
    return src[:pos] + "\n" + block + src[pos:]


def link_flags(calls) -> list:
    """Libraries the rewritten program links (from the replaced calls' records)."""
    table = load_patterns()
    flags = []
    for c in calls:
        if c.get("action", "").startswith("replaced"):
            for f in table[c["name"]]["replacement"]["link"]:
                if f not in flags:
                    flags.append(f)
    return flags


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="Replace external CPU library calls by libfb calls of the same meaning")
    ap.add_argument("source")
    ap.add_argument("-o", "--output", required=True)
    ap.add_argument("--patterns", default=PATTERNS)
    args = ap.parse_args(argv)
    table = load_patterns(args.patterns)
    with open(args.source) as f:
        src = f.read()
    out, calls = rewrite(src, table)
    with open(args.output, "w") as f:
        f.write(out)
    for c in calls:
        print("%s:%d:%d: %s (%s, %d arguments): %s" % (args.source, c["line"], c["column"], c["name"], c["library"],
                                                      len(c["args"]), c["action"]))
    return 0 if all(c["interface_ok"] for c in calls) else 3


if __name__ == "__main__":
    sys.exit(main())
