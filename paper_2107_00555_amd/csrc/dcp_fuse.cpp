// dcp_fuse.cpp -- a small fusing compiler for element-wise + stencil array
// programs: the paper's greedy subgraph fusion and transient elimination
// (Sec. 3.1) applied to programs in single-operator SSA form (the first
// translation pass of Sec. 2.3), generating HIP for gfx950 at run time.
//
// Program text, one statement per line ('#' starts a comment):
//     dtype f64 | f32
//     input  NAME ...            fields in memory (x fastest, nx*ny*nz)
//     param  NAME ...            scalars given at run time (doubles)
//     NAME = add|sub|mul|div A B
//     NAME = neg A
//     NAME = copy A
//     NAME = shift A dx dy dz    A at (x+dx, y+dy, z+dz), A a field
//     output NAME ...            fields written to memory
// An operand is a name defined above or a numeric literal.  Each statement
// is one map over the grid (or one scalar, when every operand is a scalar)
// and rounds once; shifted reads follow the boundary rule of the run
// (ghost zero, or periodic).
//
// Fusion.  Statements are placed greedily, in order, in the earliest
// kernel where their operands are available: a point-wise operand computed
// in kernel j is available in kernel j (in a register) or later (from
// memory); a shifted operand must be in memory, so a shift of a value
// computed in kernel j goes to kernel j+1 (an input is always in memory).
// A value is written to memory only if it is an output or a later kernel
// reads it (transient elimination); everything else stays in registers.
// With fusion off every statement is its own kernel and every value is
// written (the unoptimised translation).  The generated code evaluates the
// statements in program order with the library's flags (no contraction), so
// fused and unfused results are the same bit for bit.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "dcp.h"

namespace {

enum Kind { K_INPUT, K_PARAM, K_CONST, K_ADD, K_SUB, K_MUL, K_DIV, K_NEG, K_COPY, K_SHIFT };

struct Node {
    Kind kind;
    int a = -1, b = -1;           // operand node indices
    int dx = 0, dy = 0, dz = 0;   // K_SHIFT
    double cval = 0.0;            // K_CONST
    int slot = -1;                // input / param index
    bool field = true;            // per point (else a scalar)
    std::string name;
    int kernel = -1;              // fields computed in a kernel (inputs: -1)
    bool stored = false;          // written to memory
    int out = -1;                 // output index
    int buf = -1;                 // workspace buffer of a stored non-output
};

struct Kernel {
    std::vector<int> nodes;       // computed here, program order
    std::vector<int> reads;       // fields read from memory (inputs or stored)
    std::vector<int> writes;      // fields stored here
    std::string fname;
};

bool is_ident(const std::string &s) {
    if (s.empty() || !(std::isalpha((unsigned char)s[0]) || s[0] == '_')) return false;
    for (char c : s)
        if (!(std::isalnum((unsigned char)c) || c == '_')) return false;
    return true;
}

std::string hexf(double v) {
    char b[64];
    std::snprintf(b, sizeof b, "%a", v);
    return b;
}

}  // namespace

struct dcp_fused {
    int dtype = DCP_F64;
    bool fuse = true;
    std::vector<Node> nodes;
    std::vector<int> inputs, params, outputs;  // node indices in declaration order
    std::vector<Kernel> kernels;
    int nbufs = 0;
    std::string source;
    std::vector<char> code;                    // compiled code object
    std::map<int, std::pair<hipModule_t, std::vector<hipFunction_t>>> modules;  // per device
    ~dcp_fused() {
        for (auto &m : modules) hipModuleUnload(m.second.first);
    }
};

namespace {

struct Parser {
    dcp_fused *p;
    std::map<std::string, int> names;
    std::string err;

    bool fail(int line, const std::string &msg) {
        err = "line " + std::to_string(line) + ": " + msg;
        return false;
    }
    int operand(const std::string &tok, int line) {
        auto it = names.find(tok);
        if (it != names.end()) return it->second;
        char *end = nullptr;
        const double v = std::strtod(tok.c_str(), &end);
        if (end && *end == '\0' && !tok.empty() && !is_ident(tok)) {
            Node n;
            n.kind = K_CONST;
            n.cval = v;
            n.field = false;
            p->nodes.push_back(n);
            return (int)p->nodes.size() - 1;
        }
        fail(line, "undefined name or bad literal '" + tok + "'");
        return -1;
    }
    bool define(const std::string &name, int line) {
        if (!is_ident(name)) return fail(line, "bad name '" + name + "'");
        if (names.count(name)) return fail(line, "'" + name + "' is defined twice");
        return true;
    }
    bool parse(const char *text) {
        std::istringstream in(text);
        std::string raw;
        int line = 0;
        bool have_dtype = false;
        while (std::getline(in, raw)) {
            ++line;
            const size_t hash = raw.find('#');
            if (hash != std::string::npos) raw.resize(hash);
            std::istringstream ls(raw);
            std::vector<std::string> t;
            for (std::string w; ls >> w;) t.push_back(w);
            if (t.empty()) continue;
            if (t[0] == "dtype") {
                if (t.size() != 2 || (t[1] != "f64" && t[1] != "f32")) return fail(line, "dtype f64 | f32");
                p->dtype = t[1] == "f64" ? DCP_F64 : DCP_F32;
                have_dtype = true;
            } else if (t[0] == "input" || t[0] == "param") {
                const bool inp = t[0] == "input";
                for (size_t i = 1; i < t.size(); ++i) {
                    if (!define(t[i], line)) return false;
                    Node n;
                    n.kind = inp ? K_INPUT : K_PARAM;
                    n.field = inp;
                    n.name = t[i];
                    n.slot = (int)(inp ? p->inputs.size() : p->params.size());
                    p->nodes.push_back(n);
                    const int id = (int)p->nodes.size() - 1;
                    (inp ? p->inputs : p->params).push_back(id);
                    names[t[i]] = id;
                }
            } else if (t[0] == "output") {
                for (size_t i = 1; i < t.size(); ++i) {
                    auto it = names.find(t[i]);
                    if (it == names.end()) return fail(line, "output of undefined '" + t[i] + "'");
                    Node &n = p->nodes[it->second];
                    if (!n.field) return fail(line, "output '" + t[i] + "' is a scalar");
                    if (n.kind == K_INPUT) return fail(line, "output '" + t[i] + "' is an input");
                    if (n.out >= 0) return fail(line, "'" + t[i] + "' is output twice");
                    n.out = (int)p->outputs.size();
                    p->outputs.push_back(it->second);
                }
            } else {
                if (t.size() < 3 || t[1] != "=") return fail(line, "expected NAME = op ...");
                if (!define(t[0], line)) return false;
                const std::string &op = t[2];
                Node n;
                n.name = t[0];
                if (op == "add" || op == "sub" || op == "mul" || op == "div") {
                    if (t.size() != 5) return fail(line, op + " takes two operands");
                    n.kind = op == "add" ? K_ADD : op == "sub" ? K_SUB : op == "mul" ? K_MUL : K_DIV;
                    if ((n.a = operand(t[3], line)) < 0 || (n.b = operand(t[4], line)) < 0) return false;
                    n.field = p->nodes[n.a].field || p->nodes[n.b].field;
                } else if (op == "neg" || op == "copy") {
                    if (t.size() != 4) return fail(line, op + " takes one operand");
                    n.kind = op == "neg" ? K_NEG : K_COPY;
                    if ((n.a = operand(t[3], line)) < 0) return false;
                    n.field = p->nodes[n.a].field;
                } else if (op == "shift") {
                    if (t.size() != 7) return fail(line, "shift A dx dy dz");
                    n.kind = K_SHIFT;
                    if ((n.a = operand(t[3], line)) < 0) return false;
                    if (!p->nodes[n.a].field) return fail(line, "shift of a scalar");
                    int d[3];
                    for (int k = 0; k < 3; ++k) {
                        char *end = nullptr;
                        const long v = std::strtol(t[4 + k].c_str(), &end, 10);
                        if (!end || *end || v < -1000000 || v > 1000000) return fail(line, "bad shift offset");
                        d[k] = (int)v;
                    }
                    n.dx = d[0];
                    n.dy = d[1];
                    n.dz = d[2];
                    n.field = true;
                } else {
                    return fail(line, "unknown operation '" + op + "'");
                }
                p->nodes.push_back(n);
                names[t[0]] = (int)p->nodes.size() - 1;
            }
        }
        if (!have_dtype) return fail(line, "missing dtype");
        if (p->outputs.empty()) return fail(line, "no output");
        return true;
    }
};

// Greedy placement and storage decisions (see the file comment).
void plan(dcp_fused *p) {
    auto &N = p->nodes;
    int nk = 0;
    for (size_t i = 0; i < N.size(); ++i) {
        Node &n = N[i];
        if (!n.field || n.kind == K_INPUT) continue;
        int k = 0;
        auto need = [&](int o, bool shifted) {
            const Node &m = N[o];
            if (!m.field || m.kind == K_INPUT) return;
            k = std::max(k, shifted ? m.kernel + 1 : m.kernel);
        };
        if (n.a >= 0) need(n.a, n.kind == K_SHIFT);
        if (n.b >= 0) need(n.b, false);
        if (!p->fuse) k = nk;  // one statement per kernel, in order
        n.kernel = k;
        nk = std::max(nk, k + 1);
    }
    p->kernels.assign((size_t)nk, Kernel{});
    for (size_t i = 0; i < N.size(); ++i)
        if (N[i].field && N[i].kind != K_INPUT) p->kernels[(size_t)N[i].kernel].nodes.push_back((int)i);
    // a field is stored if it is an output, or read by a later kernel or by a shift
    for (size_t i = 0; i < N.size(); ++i) {
        Node &n = N[i];
        if (n.out >= 0) n.stored = true;
        if (!p->fuse && n.field && n.kind != K_INPUT) n.stored = true;
        for (int o : {n.a, n.b}) {
            if (o < 0) continue;
            Node &m = N[o];
            if (!m.field || m.kind == K_INPUT || !n.field) continue;
            if (n.kind == K_SHIFT || m.kernel != n.kernel) m.stored = true;
        }
    }
    for (auto &n : N)
        if (n.stored && n.out < 0) n.buf = p->nbufs++;
    // memory reads of each kernel: inputs and stored fields of earlier kernels
    for (size_t k = 0; k < p->kernels.size(); ++k) {
        Kernel &K = p->kernels[k];
        std::vector<char> seen(N.size(), 0);
        for (int i : K.nodes) {
            const Node &n = N[i];
            for (int o : {n.a, n.b}) {
                if (o < 0 || seen[o]) continue;
                const Node &m = N[o];
                if (!m.field) continue;
                if (m.kind == K_INPUT || m.kernel != (int)k) {
                    seen[o] = 1;
                    K.reads.push_back(o);
                }
            }
            if (n.stored) K.writes.push_back(i);
        }
        K.fname = "dcp_fused_k" + std::to_string(k);
    }
}

// Scalars are expanded where they are used (they cost a few instructions).
std::string scalar_expr(const dcp_fused *p, int i, const char *T) {
    const Node &n = p->nodes[i];
    switch (n.kind) {
        case K_PARAM: return "((" + std::string(T) + ")p" + std::to_string(n.slot) + ")";
        case K_CONST: return "((" + std::string(T) + ")" + hexf(n.cval) + ")";
        case K_NEG: return "(-" + scalar_expr(p, n.a, T) + ")";
        case K_COPY: return scalar_expr(p, n.a, T);
        default: break;
    }
    const char *op = n.kind == K_ADD ? " + " : n.kind == K_SUB ? " - " : n.kind == K_MUL ? " * " : " / ";
    // each operation rounds once: keep the statement's own rounding
    return "((" + std::string(T) + ")(" + scalar_expr(p, n.a, T) + op + scalar_expr(p, n.b, T) + "))";
}

void generate(dcp_fused *p) {
    const char *T = p->dtype == DCP_F64 ? "double" : "float";
    std::ostringstream s;
    s << "// generated by dcp_fuse\n"
      << "typedef long long i64;\n"
      << "template <typename T> __device__ __forceinline__ T dcp_ld(const T *__restrict__ a, i64 x, i64 y, "
         "i64 z, i64 nx, i64 ny, i64 nz, int bc) {\n"
      << "    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) {\n"
      << "        if (bc == 0) return T(0);\n"
      << "        x %= nx; if (x < 0) x += nx;\n"
      << "        y %= ny; if (y < 0) y += ny;\n"
      << "        z %= nz; if (z < 0) z += nz;\n"
      << "    }\n"
      << "    return a[x + nx * (y + ny * z)];\n"
      << "}\n";
    for (size_t k = 0; k < p->kernels.size(); ++k) {
        const Kernel &K = p->kernels[k];
        s << "extern \"C\" __global__ void __launch_bounds__(256) " << K.fname << "(";
        bool first = true;
        auto sep = [&]() { s << (first ? "" : ", "); first = false; };
        for (int r : K.reads) {
            sep();
            s << "const " << T << " *__restrict__ m" << r;
        }
        for (int w : K.writes) {
            sep();
            s << T << " *__restrict__ w" << w;
        }
        for (size_t j = 0; j < p->params.size(); ++j) {
            sep();
            s << "double p" << j;
        }
        sep();
        s << "i64 nx, i64 ny, i64 nz, int bc) {\n";
        s << "    const i64 n = nx * ny * nz;\n"
          << "    for (i64 i = (i64)blockIdx.x * 256 + threadIdx.x; i < n; i += (i64)gridDim.x * 256) {\n"
          << "        const i64 x = i % nx, yz = i / nx, y = yz % ny, z = yz / ny;\n"
          << "        (void)x; (void)y; (void)z;\n";
        // memory operands read point-wise, loaded once
        std::vector<char> loaded(p->nodes.size(), 0);
        auto val = [&](int o) -> std::string {
            const Node &m = p->nodes[o];
            if (!m.field) return scalar_expr(p, o, T);
            const bool mem = m.kind == K_INPUT || m.kernel != (int)k;
            if (mem) {
                if (!loaded[o]) {
                    s << "        const " << T << " r" << o << " = m" << o << "[i];\n";
                    loaded[o] = 1;
                }
                return "r" + std::to_string(o);
            }
            return "v" + std::to_string(o);
        };
        for (int i : K.nodes) {
            const Node &n = p->nodes[i];
            std::string e;
            if (n.kind == K_SHIFT) {
                e = "dcp_ld<" + std::string(T) + ">(m" + std::to_string(n.a) + ", x + (" + std::to_string(n.dx) +
                    "), y + (" + std::to_string(n.dy) + "), z + (" + std::to_string(n.dz) + "), nx, ny, nz, bc)";
            } else if (n.kind == K_NEG) {
                e = "-" + val(n.a);
            } else if (n.kind == K_COPY) {
                e = val(n.a);
            } else {
                const std::string a = val(n.a), b = val(n.b);
                const char *op = n.kind == K_ADD ? " + " : n.kind == K_SUB ? " - " : n.kind == K_MUL ? " * " : " / ";
                e = a + op + b;
            }
            s << "        const " << T << " v" << i << " = " << e << ";\n";
            if (n.stored) s << "        w" << i << "[i] = v" << i << ";\n";
        }
        s << "    }\n}\n";
    }
    p->source = s.str();
}

bool compile(dcp_fused *p, std::string *err) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, p->source.c_str(), "dcp_fused.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return false;
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        *err = "hiprtc: " + log;
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    p->code.resize(cs);
    hiprtcGetCode(prog, p->code.data());
    hiprtcDestroyProgram(&prog);
    return true;
}

void copy_err(const std::string &m, char *err, size_t errlen) {
    if (!err || errlen == 0) return;
    std::strncpy(err, m.c_str(), errlen - 1);
    err[errlen - 1] = '\0';
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

extern "C" {

int dcp_fuse_build(const char *program, int fuse, dcp_fused **out, char *err, size_t errlen) {
    if (!program || !out) return DCP_E_NULL;
    *out = nullptr;
    std::unique_ptr<dcp_fused> p(new dcp_fused);
    p->fuse = fuse != 0;
    Parser ps{p.get(), {}, {}};
    if (!ps.parse(program)) {
        copy_err(ps.err, err, errlen);
        return DCP_E_ARG;
    }
    plan(p.get());
    generate(p.get());
    std::string cerr;
    if (!compile(p.get(), &cerr)) {
        copy_err(cerr, err, errlen);
        return DCP_E_HIP;
    }
    *out = p.release();
    return DCP_OK;
}

void dcp_fuse_free(dcp_fused *p) { delete p; }

int dcp_fuse_info(const dcp_fused *p, int32_t *info, int32_t n) {
    if (!p || !info) return DCP_E_NULL;
    const int32_t v[6] = {p->dtype, (int32_t)p->inputs.size(), (int32_t)p->params.size(),
                          (int32_t)p->outputs.size(), (int32_t)p->kernels.size(), (int32_t)p->nbufs};
    for (int32_t i = 0; i < n && i < 6; ++i) info[i] = v[i];
    return DCP_OK;
}

int dcp_fuse_source(const dcp_fused *p, char *buf, size_t len, size_t *needed) {
    if (!p || !needed) return DCP_E_NULL;
    *needed = p->source.size() + 1;
    if (buf) {
        if (len < *needed) return DCP_E_WORKSPACE;
        std::memcpy(buf, p->source.c_str(), *needed);
    }
    return DCP_OK;
}

int dcp_fuse_workspace_bytes(const dcp_fused *p, int64_t nx, int64_t ny, int64_t nz, size_t *bytes) {
    if (!p || !bytes) return DCP_E_NULL;
    if (nx < 0 || ny < 0 || nz < 0) return DCP_E_SHAPE;
    const size_t esz = p->dtype == DCP_F64 ? 8 : 4;
    const int64_t lim = ((int64_t)1 << 60) / 8;
    if ((nx && ny && (nx > lim / ny || nx * ny > lim / std::max<int64_t>(nz, 1)))) return DCP_E_SHAPE;
    *bytes = (size_t)p->nbufs * align256((size_t)(nx * ny * nz) * esz);
    return DCP_OK;
}

int dcp_fuse_run(dcp_fused *p, const void *const *inputs, const double *params, void *const *outputs, int64_t nx,
                 int64_t ny, int64_t nz, int bc, void *ws, size_t ws_bytes, void *stream) {
    if (!p) return DCP_E_NULL;
    if (nx < 0 || ny < 0 || nz < 0) return DCP_E_SHAPE;
    if (bc != DCP_DIRICHLET0 && bc != DCP_PERIODIC) return DCP_E_BC;
    size_t need = 0;
    int rc = dcp_fuse_workspace_bytes(p, nx, ny, nz, &need);
    if (rc) return rc;
    const int64_t n = nx * ny * nz;
    if (n == 0) return DCP_OK;
    if (!p->inputs.empty() && !inputs) return DCP_E_NULL;
    if (!p->params.empty() && !params) return DCP_E_NULL;
    if (!outputs) return DCP_E_NULL;
    for (size_t i = 0; i < p->inputs.size(); ++i)
        if (!inputs[i]) return DCP_E_NULL;
    for (size_t i = 0; i < p->outputs.size(); ++i)
        if (!outputs[i]) return DCP_E_NULL;
    for (size_t j = 0; j < p->params.size(); ++j)
        if (!std::isfinite(params[j])) return DCP_E_ARG;
    if (need && (!ws || ws_bytes < need)) return ws ? DCP_E_WORKSPACE : DCP_E_NULL;
    const size_t fb = (size_t)n * (p->dtype == DCP_F64 ? 8 : 4);
    auto ov = [](const void *a, size_t na, const void *b, size_t nb) {
        const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
        return a && b && x < y + nb && y < x + na;
    };
    for (size_t i = 0; i < p->outputs.size(); ++i) {
        for (size_t j = 0; j < p->inputs.size(); ++j)
            if (ov(outputs[i], fb, inputs[j], fb)) return DCP_E_ALIAS;
        for (size_t j = i + 1; j < p->outputs.size(); ++j)
            if (ov(outputs[i], fb, outputs[j], fb)) return DCP_E_ALIAS;
        if (ov(outputs[i], fb, ws, need)) return DCP_E_ALIAS;
    }
    for (size_t j = 0; j < p->inputs.size(); ++j)
        if (ov(inputs[j], fb, ws, need)) return DCP_E_ALIAS;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DCP_E_HIP;
    auto it = p->modules.find(dev);
    if (it == p->modules.end()) {
        hipModule_t m;
        if (hipModuleLoadData(&m, p->code.data()) != hipSuccess) return DCP_E_HIP;
        std::vector<hipFunction_t> fns;
        for (const Kernel &K : p->kernels) {
            hipFunction_t f;
            if (hipModuleGetFunction(&f, m, K.fname.c_str()) != hipSuccess) {
                hipModuleUnload(m);
                return DCP_E_HIP;
            }
            fns.push_back(f);
        }
        it = p->modules.emplace(dev, std::make_pair(m, fns)).first;
    }
    auto ptr_of = [&](int node) -> void * {
        const Node &m = p->nodes[node];
        if (m.kind == K_INPUT) return const_cast<void *>(inputs[m.slot]);
        if (m.out >= 0) return outputs[m.out];
        return static_cast<char *>(ws) + (size_t)m.buf * align256(fb);
    };
    const int64_t blocks64 = std::min<int64_t>((n + 255) / 256, 1 << 16);
    const unsigned blocks = (unsigned)std::max<int64_t>(blocks64, 1);
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (size_t k = 0; k < p->kernels.size(); ++k) {
        const Kernel &K = p->kernels[k];
        std::vector<void *> ptrs;
        for (int r : K.reads) ptrs.push_back(ptr_of(r));
        for (int w : K.writes) ptrs.push_back(ptr_of(w));
        std::vector<double> pv(params ? params : nullptr, params ? params + p->params.size() : nullptr);
        int64_t dims[3] = {nx, ny, nz};
        int bcv = bc;
        std::vector<void *> args;
        for (auto &q : ptrs) args.push_back(&q);
        for (auto &v : pv) args.push_back(&v);
        for (auto &d : dims) args.push_back(&d);
        args.push_back(&bcv);
        if (hipModuleLaunchKernel(it->second.second[k], blocks, 1, 1, 256, 1, 1, 0, st, args.data(), nullptr) !=
            hipSuccess)
            return DCP_E_HIP;
    }
    return DCP_OK;
}

}  // extern "C"
