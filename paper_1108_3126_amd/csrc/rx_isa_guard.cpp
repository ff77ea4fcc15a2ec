// Static check of the register-staged sliced kernels.
//
// Those kernels issue their global loads from inline assembly into
// accumulation registers (AGPRs) and wait for them with explicit s_waitcnt
// before the same registers are written to LDS by inline assembly.  The
// device compiler takes an assembly output as written as soon as the
// statement ends, so any instruction of its own that read, copied or moved
// such a register between the load and the wait would see stale bytes.  The
// guard disassembles the generated code object (our own, built at run time)
// with the code-object manager's disassembler and accepts a kernel only when
// every instruction that names an AGPR is one of the two the kernels write
// themselves: the 16-byte global load (the only writer) and the 16-byte LDS
// write (the only reader).  Any compiler-made AGPR access -- a copy, a spill,
// a split live range -- rejects the kernel, and the LDS-staged kernel (loads
// tracked by the compiler) runs in its place.
#include <dlfcn.h>

#include <cctype>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rx_internal.h"

namespace rx {

namespace {

// the few code-object-manager entry points used here (resolved at run time)
typedef struct { uint64_t handle; } comgr_disasm_t;
typedef int (*create_fn)(const char*, uint64_t (*)(uint64_t, char*, uint64_t, void*), void (*)(const char*, void*),
                         void (*)(uint64_t, void*), comgr_disasm_t*);
typedef int (*disasm_fn)(comgr_disasm_t, uint64_t, void*, uint64_t*);
typedef int (*destroy_fn)(comgr_disasm_t);

struct Comgr {
    create_fn create = nullptr;
    disasm_fn disasm = nullptr;
    destroy_fn destroy = nullptr;
    bool ok = false;
};

const Comgr& comgr() {
    static Comgr C;
    static std::once_flag once;
    std::call_once(once, [] {
        void* h = nullptr;
        // prefer the copy the run-time compiler already loaded
        for (const char* name : {"libamd_comgr.so", "libamd_comgr.so.3"})
            if (!h) h = dlopen(name, RTLD_NOW | RTLD_NOLOAD);
        for (const char* name : {"libamd_comgr.so.3", "libamd_comgr.so"})
            if (!h) h = dlopen(name, RTLD_NOW);
        if (!h) return;
        C.create = reinterpret_cast<create_fn>(dlsym(h, "amd_comgr_create_disassembly_info"));
        C.disasm = reinterpret_cast<disasm_fn>(dlsym(h, "amd_comgr_disassemble_instruction"));
        C.destroy = reinterpret_cast<destroy_fn>(dlsym(h, "amd_comgr_destroy_disassembly_info"));
        C.ok = C.create && C.disasm && C.destroy;
    });
    return C;
}

// ELF64 little-endian structures (the AMDGPU code object format)
struct Ehdr {
    unsigned char ident[16];
    uint16_t type, machine;
    uint32_t version;
    uint64_t entry, phoff, shoff;
    uint32_t flags;
    uint16_t ehsize, phentsize, phnum, shentsize, shnum, shstrndx;
};
struct Shdr {
    uint32_t name, type;
    uint64_t flags, addr, offset, size;
    uint32_t link, info;
    uint64_t addralign, entsize;
};
struct Sym {
    uint32_t name;
    unsigned char info, other;
    uint16_t shndx;
    uint64_t value, size;
};

// File range [off, off + size) of function `name`, or false.
bool find_function(const std::vector<char>& elf, const char* name, uint64_t* off, uint64_t* size) {
    if (elf.size() < sizeof(Ehdr) || std::memcmp(elf.data(), "\x7f" "ELF", 4) != 0 || elf[4] != 2) return false;
    Ehdr eh;
    std::memcpy(&eh, elf.data(), sizeof(eh));
    if (eh.shentsize != sizeof(Shdr) || eh.shoff + (uint64_t)eh.shnum * sizeof(Shdr) > elf.size()) return false;
    std::vector<Shdr> sh(eh.shnum);
    std::memcpy(sh.data(), elf.data() + eh.shoff, sizeof(Shdr) * eh.shnum);
    for (const Shdr& s : sh) {
        if (s.type != 2 /* SHT_SYMTAB */ || s.link >= sh.size() || s.entsize != sizeof(Sym)) continue;
        const Shdr& strtab = sh[s.link];
        if (s.offset + s.size > elf.size() || strtab.offset + strtab.size > elf.size()) return false;
        for (uint64_t k = 0; k < s.size / sizeof(Sym); ++k) {
            Sym y;
            std::memcpy(&y, elf.data() + s.offset + k * sizeof(Sym), sizeof(y));
            if ((y.info & 0xf) != 2 /* STT_FUNC */ || y.name >= strtab.size || y.shndx >= sh.size()) continue;
            const char* nm = elf.data() + strtab.offset + y.name;
            if (std::strncmp(nm, name, strtab.size - y.name) != 0 || std::strlen(name) != strnlen(nm, strtab.size - y.name))
                continue;
            const Shdr& sec = sh[y.shndx];
            if (y.value < sec.addr || y.value + y.size > sec.addr + sec.size) return false;
            *off = y.value - sec.addr + sec.offset;
            *size = y.size;
            return *off + *size <= elf.size();
        }
    }
    return false;
}

struct Walk {
    const std::vector<char>* elf;
    std::string text;   // the instruction just printed
};

uint64_t read_cb(uint64_t from, char* to, uint64_t size, void* user) {
    const Walk* w = static_cast<const Walk*>(user);
    if (from >= w->elf->size()) return 0;
    const uint64_t n = std::min<uint64_t>(size, w->elf->size() - from);
    std::memcpy(to, w->elf->data() + from, n);
    return n;
}
void print_cb(const char* ins, void* user) { static_cast<Walk*>(user)->text = ins; }
void annot_cb(uint64_t, void*) {}

// Does the operand text name an accumulation register (a5, a[4:7])?
bool names_agpr(const std::string& ops) {
    for (size_t i = 0; i < ops.size(); ++i) {
        if (ops[i] != 'a') continue;
        const bool start = i == 0 || !(std::isalnum((unsigned char)ops[i - 1]) || ops[i - 1] == '_');
        if (start && i + 1 < ops.size() && (std::isdigit((unsigned char)ops[i + 1]) || ops[i + 1] == '[')) return true;
    }
    return false;
}

}  // namespace

int isa_check_agpr_staging(const std::vector<char>& code, const std::string& arch, const char* kernel,
                           int* violations, std::string* example) {
    *violations = 0;
    const Comgr& C = comgr();
    if (!C.ok) return -1;
    uint64_t off = 0, size = 0;
    if (!find_function(code, kernel, &off, &size)) return -2;
    const std::string isa = "amdgcn-amd-amdhsa--" + arch;
    comgr_disasm_t info{0};
    if (C.create(isa.c_str(), read_cb, print_cb, annot_cb, &info) != 0) return -3;
    Walk w{&code, {}};
    int rc = 0;
    int own = 0;   // instructions of the kernel's own staging that name an AGPR
    for (uint64_t a = off; a < off + size;) {
        uint64_t used = 0;
        w.text.clear();
        if (C.disasm(info, a, &w, &used) != 0 || used == 0) {
            rc = -4;
            break;
        }
        a += used;
        size_t p = w.text.find_first_not_of(" \t");
        if (p == std::string::npos) continue;
        const size_t q = w.text.find_first_of(" \t", p);
        const std::string mnem = w.text.substr(p, q == std::string::npos ? std::string::npos : q - p);
        const std::string ops = q == std::string::npos ? std::string() : w.text.substr(q);
        if (!names_agpr(ops)) continue;
        if (mnem == "global_load_dwordx4" || mnem == "ds_write_b128") {
            ++own;
            continue;
        }
        if (++*violations == 1 && example) *example = w.text;
    }
    C.destroy(info);
    // a staged kernel always holds its own AGPR loads and writes; seeing none
    // means the text was not understood, and the check has not run
    if (rc == 0 && own == 0) rc = -5;
    return rc;
}

}  // namespace rx
