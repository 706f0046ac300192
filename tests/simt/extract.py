"""Copy top-level definitions (functions by name, `const:NAME` for constexpr lines,
`struct:NAME` for a struct or struct template) out of a kernel source file, so that the CPU
harness compiles the current kernel text.

    python extract.py <source.hip> NAME... > out.inc
"""
import re, sys
src = open(sys.argv[1]).read()
names = sys.argv[2:]
lines = src.split("\n")
out = []
def grab_function(name):
    for i, l in enumerate(lines):
        if re.search(r"\b" + re.escape(name) + r"\s*\(", l) and (l.startswith("__global__") or l.startswith("__device__")):
            start = i
            if i > 0 and lines[i - 1].startswith("template"):
                start = i - 1
            text = "\n".join(lines[start:])
            # from the first '{' after the signature, match braces
            k = text.index("{", len("\n".join(lines[start:i + 1])) - len(lines[i]))
            depth = 0
            for q in range(k, len(text)):
                c = text[q]
                if c == "{": depth += 1
                elif c == "}":
                    depth -= 1
                    if depth == 0:
                        return text[:q + 1]
    raise SystemExit(f"not found: {name}")
def grab_struct(name):
    for i, l in enumerate(lines):
        if re.match(r"^struct " + re.escape(name) + r"\b", l):
            start = i - 1 if i > 0 and lines[i - 1].startswith("template") else i
            end = i
            while not lines[end].startswith("};"):
                end += 1
            return "\n".join(lines[start:end + 1])
    raise SystemExit(f"struct not found: {name}")
for n in names:
    if n.startswith("struct:"):
        out.append(grab_struct(n[7:]))
    elif n.startswith("const:"):
        nm = n[6:]
        hit = [l for l in lines if re.match(r"^constexpr .*\b" + re.escape(nm) + r"\b\s*=", l)]
        if not hit: raise SystemExit(f"const not found: {nm}")
        out.append(hit[0])
    else:
        out.append(grab_function(n))
print("\n\n".join(out))
