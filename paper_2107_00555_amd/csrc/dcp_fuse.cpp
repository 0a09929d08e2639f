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

#include <algorithm>
#include <cctype>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "dcp.h"
#include "dcp_internal.h"

namespace {

constexpr int kRows = 4;  // waves (rows) per workgroup (8 measured slightly slower)

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
    std::mutex modules_mu;                     // guards modules (runs from several threads)
    ~dcp_fused() {
        // runs may still be in flight: wait for each device that holds the
        // code before unloading it
        int cur = 0;
        const bool have_cur = hipGetDevice(&cur) == hipSuccess;
        for (auto &m : modules) {
            if (hipSetDevice(m.first) == hipSuccess) (void)hipDeviceSynchronize();
            hipModuleUnload(m.second.first);
        }
        if (have_cur && !modules.empty()) (void)hipSetDevice(cur);
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
            if (!std::isfinite(v)) {
                fail(line, "literal '" + tok + "' is not a finite double");
                return -1;
            }
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
        // named by dtype and mode, so profiles tell the programs apart
        K.fname = std::string("dcp_gen_") + (p->dtype == DCP_F64 ? "f64" : "f32") + (p->fuse ? "_fused" : "_unfused") +
                  "_k" + std::to_string(k);
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

// Generated code.  A lane computes V consecutive x-points (16 bytes of the
// dtype); a wave covers 64*V consecutive x of one (y, z) row (a wave tile)
// and walks zr planes; a workgroup takes the same x tile of four
// consecutive rows (a wave's y-neighbour rows are its siblings' rows, so
// they tend to hit the CU's cache).  y and z are uniform over a wave.  The index type is 32-bit when the grid allows
// it (a second entry point uses 64-bit indices).
//
// Reads of a memory field are grouped by (field, dy).  A group keeps, in
// registers, one aligned V-wide vector of the lane's own x-points for each
// plane z+dz its reads need (a queue that moves up one plane per step), so
// a plane costs one vector load per group, issued one plane ahead.  y and z
// wrap; under the ghost-zero rule a slot outside the grid reads as zero.  A
// read shifted by |dx| <= V takes its values from the lane's own vector and
// the neighbouring lane's (cross-lane moves).  Lanes whose values would come
// from outside the wave tile or the row (the first lane for dx < 0, the last
// lanes for dx > 0, the lane at a ragged row end), and every lane of a read
// with |dx| > V, take them per point through the boundary rule instead.
// Grids too small for one wrap per axis take every point through the rule.
// Points past the row end are computed but not stored.  The V points of a
// lane are evaluated independently, each statement rounding once, so the
// results do not depend on V or on the path taken.
void generate(dcp_fused *p) {
    const char *T = p->dtype == DCP_F64 ? "double" : "float";
    const int V = p->dtype == DCP_F64 ? 2 : 4;
    std::ostringstream s;
    s << "// generated by dcp_fuse\n"
      << "typedef long long i64;\n"
      << "#define V " << V << "\n"
      // one point through the boundary rule (the small-grid path: out of line)
      << "template <typename T, typename I> __device__ __attribute__((noinline)) T dcp_ld(const T *__restrict__ a, "
         "I x, I y, I z, I nx, I ny, I nz, int bc) {\n"
      << "    if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) {\n"
      << "        if (bc == 0) return T(0);\n"
      << "        x %= nx; if (x < 0) x += nx;\n"
      << "        y %= ny; if (y < 0) y += ny;\n"
      << "        z %= nz; if (z < 0) z += nz;\n"
      << "    }\n"
      << "    return a[x + nx * (y + ny * z)];\n"
      << "}\n"
      << "template <typename I> __device__ __forceinline__ I dcp_wrap(I c, I n) {\n"
      << "    return c < 0 ? c + n : (c >= n ? c - n : c);\n"
      << "}\n"
      << "template <typename I> __device__ __forceinline__ bool dcp_in(I c, I n) { return c >= 0 && c < n; }\n"
      // r = this lane's bit of the wave mask m set ? a : b; taking the
      // choice from the mask keeps the optimiser from merging the two
      // sources into one register (which would make a vector load wait)
      << "__device__ __forceinline__ unsigned dcp_sel32(unsigned long long m, unsigned a, unsigned b) {\n"
      << "    const unsigned lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));\n"
      << "    return ((m >> lane) & 1ull) ? a : b;\n"
      << "}\n"
      << "__device__ __forceinline__ float dcp_sel(unsigned long long m, float a, float b) {\n"
      << "    return __builtin_bit_cast(float, dcp_sel32(m, __builtin_bit_cast(unsigned, a), "
         "__builtin_bit_cast(unsigned, b)));\n"
      << "}\n"
      << "__device__ __forceinline__ double dcp_sel(unsigned long long m, double a, double b) {\n"
      << "    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a), "
         "ub = __builtin_bit_cast(unsigned long long, b);\n"
      << "    const unsigned long long lo = dcp_sel32(m, (unsigned)ua, (unsigned)ub);\n"
      << "    const unsigned long long hi = dcp_sel32(m, (unsigned)(ua >> 32), (unsigned)(ub >> 32));\n"
      << "    return __builtin_bit_cast(double, (hi << 32) | lo);\n"
      << "}\n"
      // the value of lane - 1 (lower) or lane + 1 (upper); zero at the wave's
      // ends and from inactive lanes
      << "template <int CTRL> __device__ __forceinline__ float dcp_dpp(float v) {\n"
      << "    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, "
         "true));\n"
      << "}\n"
      << "template <int CTRL> __device__ __forceinline__ double dcp_dpp(double v) {\n"
      << "    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);\n"
      << "    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);\n"
      << "    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);\n"
      << "    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);\n"
      << "}\n"
      << "#define DCP_LOWER 0x138\n"  // wave_shr:1
      << "#define DCP_UPPER 0x130\n"  // wave_shl:1
      // NT: the streaming (non-temporal) hint, for data a kernel touches once
      // (a field read only unshifted, every store), so that the rows a
      // shifted read fetches stay in L2 for the neighbouring tiles
      << "template <typename T, bool NT = false> __device__ __forceinline__ void dcp_ldv(const T *__restrict__ a, "
         "T *o) {\n"
      << "    typedef T vt __attribute__((ext_vector_type(V), aligned(sizeof(T))));\n"
      << "    vt v;\n"
      << "    if constexpr (NT) v = __builtin_nontemporal_load(reinterpret_cast<const vt *>(a));\n"
      << "    else __builtin_memcpy(&v, a, sizeof(vt));\n"
      << "#pragma unroll\n"
      << "    for (int j = 0; j < V; ++j) o[j] = v[j];\n"
      << "}\n"
      << "template <typename T> __device__ __forceinline__ void dcp_stv(T *__restrict__ a, const T *o) {\n"
      << "    typedef T vt __attribute__((ext_vector_type(V), aligned(sizeof(T))));\n"
      << "    vt v;\n"
      << "#pragma unroll\n"
      << "    for (int j = 0; j < V; ++j) v[j] = o[j];\n"
      << "    __builtin_nontemporal_store(v, reinterpret_cast<vt *>(a));\n"
      << "}\n"
      << "template <typename T, typename I> __device__ __forceinline__ void dcp_wr(T *__restrict__ a, "
         "const T *o, I i, I x, I nx) {\n"
      << "    if (x + V <= nx) { dcp_stv<T>(a + i, o); return; }\n"
      << "#pragma unroll\n"
      << "    for (int j = 0; j < V; ++j)\n"
      << "        if (x + j < nx) a[i + j] = o[j];\n"
      << "}\n"
      // one queue slot: the lane's V x-points of row yy, plane zz (wrapped;
      // the start clamped into the row); returns whether it reads as data
      << "template <typename T, typename I, bool NT = false> __device__ __forceinline__ bool dcp_slot(const T "
         "*__restrict__ a, T *q, I xc, I yy, I zz, I nx, I ny, I nz, int bc) {\n"
      << "    dcp_ldv<T, NT>(a + (xc + nx * (dcp_wrap<I>(yy, ny) + ny * dcp_wrap<I>(zz, nz))), q);\n"
      << "    return bc != 0 || (dcp_in<I>(yy, ny) && dcp_in<I>(zz, nz));\n"
      << "}\n"
      // V points (x + j + dx, yy, zz) through the boundary rule, one wrap
      // per axis at most; f holds zeros on entry
      << "template <typename T, typename I> __device__ __forceinline__ void dcp_fixel(const T *__restrict__ a, T *f, "
         "I x, I dx, I yy, I zz, I nx, I ny, I nz, int bc) {\n"
      << "    const bool inyz = dcp_in<I>(yy, ny) && dcp_in<I>(zz, nz);\n"
      << "    const I row = nx * (dcp_wrap<I>(yy, ny) + ny * dcp_wrap<I>(zz, nz));\n"
      << "#pragma unroll\n"
      << "    for (int j = 0; j < V; ++j) {\n"
      << "        const I xe = x + j + dx;\n"
      << "        if (bc != 0 || (inyz && dcp_in<I>(xe, nx))) f[j] = a[row + dcp_wrap<I>(xe, nx)];\n"
      << "    }\n"
      << "}\n";
    for (size_t k = 0; k < p->kernels.size(); ++k) {
        const Kernel &K = p->kernels[k];
        std::ostringstream params_decl, params_pass;
        bool first = true;
        auto sep = [&]() {
            if (!first) {
                params_decl << ", ";
                params_pass << ", ";
            }
            first = false;
        };
        for (int r : K.reads) {
            sep();
            params_decl << "const " << T << " *__restrict__ m" << r;
            params_pass << "m" << r;
        }
        for (int w : K.writes) {
            sep();
            params_decl << T << " *__restrict__ w" << w;
            params_pass << "w" << w;
        }
        for (size_t j = 0; j < p->params.size(); ++j) {
            sep();
            params_decl << "double p" << j;
            params_pass << "p" << j;
        }
        sep();
        params_decl << "i64 nx_, i64 ny_, i64 nz_, int bc";
        params_pass << "nx_, ny_, nz_, bc";

        // the kernel's memory reads (program order) and their groups
        struct Rd {
            std::string dst;
            int field, dx, dy, dz, grp;
        };
        struct Grp {
            int field, dy, dzlo, dzhi;
        };
        std::vector<Rd> rds;
        std::vector<Grp> grps;
        std::vector<char> loaded(p->nodes.size(), 0);
        auto add_read = [&](const std::string &dst, int field, int dx, int dy, int dz) {
            int g = -1;
            for (size_t q = 0; q < grps.size(); ++q)
                if (grps[q].field == field && grps[q].dy == dy) g = (int)q;
            if (g < 0) {
                grps.push_back(Grp{field, dy, dz, dz});
                g = (int)grps.size() - 1;
            }
            grps[g].dzlo = std::min(grps[g].dzlo, dz);
            grps[g].dzhi = std::max(grps[g].dzhi, dz);
            rds.push_back(Rd{dst, field, dx, dy, dz, g});
        };
        for (int i : K.nodes) {
            const Node &n = p->nodes[i];
            if (n.kind == K_SHIFT) {
                add_read("v" + std::to_string(i), n.a, n.dx, n.dy, n.dz);
                continue;
            }
            for (int o : {n.a, n.b}) {
                if (o < 0) continue;
                const Node &m = p->nodes[o];
                if (!m.field || loaded[o] || !(m.kind == K_INPUT || m.kernel != (int)k)) continue;
                add_read("r" + std::to_string(o), o, 0, 0, 0);
                loaded[o] = 1;
            }
        }
        // a group streams (non-temporal loads) when every read of its field
        // in this kernel is unshifted: no other tile or plane needs its lines
        std::vector<char> streamed(grps.size(), 1);
        for (const Rd &r : rds)
            if (r.dx != 0 || r.dy != 0 || r.dz != 0)
                for (size_t g = 0; g < grps.size(); ++g)
                    if (grps[g].field == r.field) streamed[g] = 0;
        auto slot_fn = [&](size_t g) -> std::string {
            return std::string("dcp_slot<") + T + ", I" + (streamed[g] ? ", true" : "") + ">";
        };
        int maxd[3] = {0, 0, 0};
        for (const Rd &r : rds) {
            maxd[0] = std::max(maxd[0], std::abs(r.dx));
            maxd[1] = std::max(maxd[1], std::abs(r.dy));
            maxd[2] = std::max(maxd[2], std::abs(r.dz));
        }

        // the statements and stores of one plane, given every read's values
        std::ostringstream rd_decl, rd_pass;
        for (const Rd &r : rds) {
            rd_decl << ", const " << T << " *" << r.dst;
            rd_pass << ", " << r.dst;
        }
        s << "template <typename I> __device__ __forceinline__ void " << K.fname << "_comp(" << params_decl.str()
          << ", I i, I x, I nx" << rd_decl.str() << ") {\n";
        auto val = [&](int o) -> std::string {
            const Node &m = p->nodes[o];
            if (!m.field) return scalar_expr(p, o, T);
            if (m.kind == K_INPUT || m.kernel != (int)k) return "r" + std::to_string(o) + "[j]";
            return "v" + std::to_string(o) + "[j]";
        };
        for (int i : K.nodes) {
            const Node &n = p->nodes[i];
            if (n.kind != K_SHIFT) {
                std::string e;
                if (n.kind == K_NEG) {
                    e = "-" + val(n.a);
                } else if (n.kind == K_COPY) {
                    e = val(n.a);
                } else {
                    const std::string a = val(n.a), b = val(n.b);
                    const char *op =
                        n.kind == K_ADD ? " + " : n.kind == K_SUB ? " - " : n.kind == K_MUL ? " * " : " / ";
                    e = a + op + b;
                }
                s << "    " << T << " v" << i << "[V];\n"
                  << "#pragma unroll\n"
                  << "    for (int j = 0; j < V; ++j) v" << i << "[j] = " << e << ";\n";
            }
            if (n.stored) s << "    dcp_wr<" << T << ", I>(w" << i << ", v" << i << ", i, x, nx);\n";
        }
        s << "}\n";

        // one plane, every point through the boundary rule (small grids)
        s << "template <typename I> __device__ __forceinline__ void " << K.fname << "_slow(" << params_decl.str()
          << ", I x, I y, I z, I i, I nx, I ny, I nz) {\n";
        for (const Rd &r : rds)
            s << "    " << T << " " << r.dst << "[V];\n"
              << "#pragma unroll\n"
              << "    for (int j = 0; j < V; ++j) " << r.dst << "[j] = dcp_ld<" << T << ", I>(m" << r.field
              << ", x + j + (" << r.dx << "), y + (" << r.dy << "), z + (" << r.dz << "), nx, ny, nz, bc);\n";
        s << "    " << K.fname << "_comp<I>(" << params_pass.str() << ", i, x, nx" << rd_pass.str() << ");\n"
          << "}\n";

        for (const char *suffix : {"_i32", "_i64"}) {
            const char *I = suffix[2] == '3' ? "int" : "i64";
            std::ostringstream b;  // the fast path's per-tile code
            // queue slots: Q<g>_<k> holds plane z + dzlo + k; P<g> the next top
            for (size_t g = 0; g < grps.size(); ++g) {
                const int span = grps[g].dzhi - grps[g].dzlo + 1;
                for (int q = 0; q < span; ++q)
                    b << "        " << T << " Q" << g << "_" << q << "[V];\n"
                      << "        bool W" << g << "_" << q << " = " << slot_fn(g) << "(m" << grps[g].field << ", Q"
                      << g << "_" << q << ", xc, y + (" << grps[g].dy << "), zb + (" << grps[g].dzlo + q
                      << "), nx, ny, nz, bc);\n";
                b << "        " << T << " P" << g << "[V];\n";
            }
            b << "        for (I z = zb; z < ze; ++z, i += plane) {\n"
              // a lane past a ragged row end (V points not all in the row)
              << "            const bool rg = x + V > nx;\n"
              << "            const unsigned long long mrg = __builtin_amdgcn_ballot_w64(rg);\n";
            // per read: the elements from outside the lane at a wave or row
            // end (one load each, into scalars of their own), and, in a wave
            // with a ragged lane, that lane's points through the rule
            for (size_t r = 0; r < rds.size(); ++r) {
                const Rd &R = rds[r];
                const std::string yz = "y + (" + std::to_string(R.dy) + "), z + (" + std::to_string(R.dz) + ")";
                if (std::abs(R.dx) > V) {
                    b << "            " << T << " f" << r << "[V];\n"
                      << "#pragma unroll\n"
                      << "            for (int j = 0; j < V; ++j) f" << r << "[j] = " << T << "(0);\n"
                      << "            dcp_fixel<" << T << ", I>(m" << R.field << ", f" << r << ", x, (I)(" << R.dx
                      << "), " << yz << ", nx, ny, nz, bc);\n";
                    continue;
                }
                if (R.dx != 0) {
                    const std::string ne = R.dx < 0 ? "lane == 0" : "lane == 63 || x + 2 * V > nx";
                    b << "            const bool ne" << r << " = " << ne << ";\n";
                    for (int j = 0; j < V; ++j) {
                        const int e = j + R.dx;
                        if (e >= 0 && e < V) continue;
                        b << "            " << T << " e" << r << "_" << j << " = " << T << "(0);\n";
                    }
                    b << "            if (ne" << r << ") {\n"
                      << "                const I yy = y + (" << R.dy << "), zz = z + (" << R.dz << ");\n"
                      << "                const bool inyz = dcp_in<I>(yy, ny) && dcp_in<I>(zz, nz);\n"
                      << "                const I row = nx * (dcp_wrap<I>(yy, ny) + ny * dcp_wrap<I>(zz, nz));\n";
                    for (int j = 0; j < V; ++j) {
                        const int e = j + R.dx;
                        if (e >= 0 && e < V) continue;
                        b << "                { const I xe = x + " << e << "; if (bc != 0 || (inyz && dcp_in<I>(xe, nx))) e"
                          << r << "_" << j << " = m" << R.field << "[row + dcp_wrap<I>(xe, nx)]; }\n";
                    }
                    b << "            }\n";
                }
                b << "            " << T << " g" << r << "[V];\n"
                  << "#pragma unroll\n"
                  << "            for (int j = 0; j < V; ++j) g" << r << "[j] = " << T << "(0);\n"
                  << "            if (mrg != 0 && rg) dcp_fixel<" << T << ", I>(m" << R.field << ", g" << r << ", x, (I)("
                  << R.dx << "), " << yz << ", nx, ny, nz, bc);\n";
            }
            // the next plane's top slot of every group, on every path (loads
            // complete in order: the per-point loads above go out first, so
            // waiting for them does not wait for these)
            for (size_t g = 0; g < grps.size(); ++g)
                b << "            const bool WP" << g << " = " << slot_fn(g) << "(m" << grps[g].field << ", P" << g
                  << ", xc, y + (" << grps[g].dy << "), z + (" << grps[g].dzhi + 1 << "), nx, ny, nz, bc);\n";
            // each read from its slot: element j is element j + dx of this
            // lane's vector, or of the lower / upper lane's.  In a wave with no
            // ragged lane whose slots all read as data (every periodic plane,
            // and every interior one) only the row-end elements need a choice.
            for (size_t r = 0; r < rds.size(); ++r) b << "            " << T << " " << rds[r].dst << "[V];\n";
            std::string allw = "mrg == 0";
            for (size_t g = 0; g < grps.size(); ++g) {
                const int span = grps[g].dzhi - grps[g].dzlo + 1;
                for (int q = 0; q < span; ++q) allw += " && W" + std::to_string(g) + "_" + std::to_string(q);
            }
            for (int general = 0; general < 2; ++general) {
                b << (general ? "            } else {\n" : "            if (" + allw + ") {\n");
                for (size_t r = 0; r < rds.size(); ++r) {
                    const Rd &R = rds[r];
                    const std::string slot =
                        "Q" + std::to_string(R.grp) + "_" + std::to_string(R.dz - grps[R.grp].dzlo);
                    const std::string valid =
                        "W" + std::to_string(R.grp) + "_" + std::to_string(R.dz - grps[R.grp].dzlo);
                    if (std::abs(R.dx) > V) {
                        b << "#pragma unroll\n"
                          << "                for (int j = 0; j < V; ++j) " << R.dst << "[j] = f" << r << "[j];\n";
                        continue;
                    }
                    b << "                {\n";
                    if (R.dx != 0)
                        b << "                    const unsigned long long mne = __builtin_amdgcn_ballot_w64(ne" << r
                          << ");\n";
                    for (int j = 0; j < V; ++j) {
                        const int e = j + R.dx;
                        std::string src;
                        if (e < 0)
                            src = "dcp_dpp<DCP_LOWER>(" + slot + "[" + std::to_string(e + V) + "])";
                        else if (e >= V)
                            src = "dcp_dpp<DCP_UPPER>(" + slot + "[" + std::to_string(e - V) + "])";
                        else
                            src = slot + "[" + std::to_string(e) + "]";
                        std::string c = general ? "(" + valid + " ? " + src + " : " + T + "(0))" : src;
                        if (e < 0 || e >= V)
                            c = "dcp_sel(mne, e" + std::to_string(r) + "_" + std::to_string(j) + ", " + c + ")";
                        if (general) c = "dcp_sel(mrg, g" + std::to_string(r) + "[" + std::to_string(j) + "], " + c + ")";
                        b << "                    " << R.dst << "[" << j << "] = " << c << ";\n";
                    }
                    b << "                }\n";
                }
            }
            b << "            }\n";
            b << "            " << K.fname << "_comp<I>(" << params_pass.str() << ", i, x, nx" << rd_pass.str()
              << ");\n";
            // the queues move up one plane
            for (size_t g = 0; g < grps.size(); ++g) {
                const int span = grps[g].dzhi - grps[g].dzlo + 1;
                for (int q = 0; q + 1 < span; ++q)
                    b << "#pragma unroll\n"
                      << "            for (int j = 0; j < V; ++j) Q" << g << "_" << q << "[j] = Q" << g << "_" << q + 1
                      << "[j];\n"
                      << "            W" << g << "_" << q << " = W" << g << "_" << q + 1 << ";\n";
                b << "#pragma unroll\n"
                  << "            for (int j = 0; j < V; ++j) Q" << g << "_" << span - 1 << "[j] = P" << g << "[j];\n"
                  << "            W" << g << "_" << span - 1 << " = WP" << g << ";\n";
            }
            b << "        }\n";

            s << "extern \"C\" __global__ void __launch_bounds__(" << 64 * kRows << ") " << K.fname << suffix << "("
              << params_decl.str() << ", int zr, i64 tiles_x_, i64 nchunk_) {\n"
              << "    typedef " << I << " I;\n"
              << "    const I nx = (I)nx_, ny = (I)ny_, nz = (I)nz_, tiles_x = (I)tiles_x_;\n"
              << "    const I nyb = (ny + " << kRows - 1 << ") / " << kRows << ", nwg = tiles_x * nyb * (I)nchunk_;\n"
              << "    const I G = (I)gridDim.x, bk = (I)blockIdx.x;\n"
              // workgroups go to the 8 XCDs in turn: give each XCD one
              // contiguous range of tiles so row neighbours share its L2
              << "    const I xcd = bk % 8, kq = bk / 8, q = G / 8, r = G % 8;\n"
              << "    const I lb = xcd < r ? xcd * (q + 1) + kq : r * (q + 1) + (xcd - r) * q + kq;\n"
              << "    const I wv = (I)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));\n"
              << "    const I lane = (I)(threadIdx.x & 63);\n"
              << "    const I plane = nx * ny;\n"
              // one wrap per axis reaches every neighbour
              << "    const bool fast = nx >= V + " << maxd[0] << " && ny >= " << maxd[1] << " && nz > " << maxd[2]
              << ";\n"
              // a workgroup's four waves take four consecutive rows of one x
              // tile, so a wave's y-neighbour rows are its siblings' rows
              << "    for (I L = lb; L < nwg; L += G) {\n"
              << "        const I xt = L % tiles_x, t = L / tiles_x, y = (t % nyb) * " << kRows
              << " + wv, zb = (t / nyb) * (I)zr;\n"
              << "        if (y >= ny) continue;\n"
              << "        const I x = xt * " << 64 * V << " + lane * V;\n"
              << "        if (x >= nx) continue;\n"
              << "        const I ze = (zb + (I)zr < nz ? zb + (I)zr : nz);\n"
              << "        I i = x + nx * y + plane * zb;\n"
              << "        if (!fast) {\n"
              << "            for (I z = zb; z < ze; ++z, i += plane)\n"
              << "                " << K.fname << "_slow<I>(" << params_pass.str() << ", x, y, z, i, nx, ny, nz);\n"
              << "            continue;\n"
              << "        }\n"
              << "        const I xc = x + V <= nx ? x : nx - V;\n"
              << b.str() << "    }\n"
              << "}\n";
        }
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
    std::unique_lock<std::mutex> lock(p->modules_mu);
    auto it = p->modules.find(dev);
    if (it == p->modules.end()) {
        hipModule_t m;
        if (hipModuleLoadData(&m, p->code.data()) != hipSuccess) return DCP_E_HIP;
        std::vector<hipFunction_t> fns;  // per kernel: 32-bit, then 64-bit indices
        for (const Kernel &K : p->kernels) {
            for (const char *suffix : {"_i32", "_i64"}) {
                hipFunction_t f;
                if (hipModuleGetFunction(&f, m, (K.fname + suffix).c_str()) != hipSuccess) {
                    hipModuleUnload(m);
                    return DCP_E_HIP;
                }
                fns.push_back(f);
            }
        }
        it = p->modules.emplace(dev, std::make_pair(m, fns)).first;
    }
    const std::vector<hipFunction_t> &fns = it->second.second;  // stable once inserted
    lock.unlock();
    auto ptr_of = [&](int node) -> void * {
        const Node &m = p->nodes[node];
        if (m.kind == K_INPUT) return const_cast<void *>(inputs[m.slot]);
        if (m.out >= 0) return outputs[m.out];
        return static_cast<char *>(ws) + (size_t)m.buf * align256(fb);
    };
    // wave tiles: 64*V x-points of one row (V points per lane, 16 bytes) over
    // zr consecutive planes; a workgroup takes one x tile of four consecutive
    // rows, workgroups ordered x tile, then row block, then plane chunk; a
    // one-dimensional grid of at most 2^20 workgroups strides over them.  zr
    // doubles, up to 16, while at least 4096 workgroups (16 per CU) remain.
    const int64_t tile_w = p->dtype == DCP_F64 ? 128 : 256;
    int64_t tiles_x = (nx + tile_w - 1) / tile_w;
    int64_t zr = 1;
    while (zr < 16 && tiles_x * ny * ((nz + 2 * zr - 1) / (2 * zr)) >= 4 * 4096) zr *= 2;
    if (const char *e = dcp::tuning_env("DCP_FUSE_ZR")) {  // tuning override: planes per wave tile
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 1 && v <= 4096) zr = v;
    }
    int64_t nchunk = (nz + zr - 1) / zr;
    const unsigned grid = (unsigned)std::min<int64_t>(tiles_x * ((ny + kRows - 1) / kRows) * nchunk, 1 << 20);
    int zr32 = (int)zr;
    double smax[3] = {0, 0, 0};  // largest |offset| of any shifted read, per axis
    for (const Node &m : p->nodes)
        if (m.kind == K_SHIFT) {
            smax[0] = std::max(smax[0], (double)std::abs(m.dx));
            smax[1] = std::max(smax[1], (double)std::abs(m.dy));
            smax[2] = std::max(smax[2], (double)std::abs(m.dz));
        }
    // every 32-bit intermediate (a point's index, an offset neighbour's
    // index, a coordinate plus an offset, a tile start rounded up to 256, a
    // row or chunk start one grid stride past the end) is bounded by this sum
    const bool idx32 = 2.0 * (double)n + smax[0] + (double)nx * (smax[1] + (double)ny * smax[2]) +
                           (double)(1 << 21) <
                       (double)INT32_MAX;
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
        args.push_back(&zr32);
        args.push_back(&tiles_x);
        args.push_back(&nchunk);
        hipFunction_t fn = fns[2 * k + (idx32 ? 0 : 1)];
        if (hipModuleLaunchKernel(fn, grid, 1, 1, 64 * kRows, 1, 1, 0, st, args.data(),
                                  nullptr) != hipSuccess)
            return DCP_E_HIP;
    }
    return DCP_OK;
}

}  // extern "C"
