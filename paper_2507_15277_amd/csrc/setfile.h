// Host-only parsing of variant descriptors, manifests and variant-set files
// (the offline output of portability tuning that the runtime loads, Fig. 1).
// No HIP types: the parser builds and runs on its own.
#pragma once

#include <array>
#include <cstdint>
#include <istream>
#include <string>
#include <vector>

constexpr int kFfPrecForms = 5;    // precision forms of a variant (FF_FORM_FP32 .. FF_FORM_FP16X3)
constexpr int kFfForms = 6;        // set slots: the precision forms and FF_FORM_MIXED
constexpr int kFfMaxMembers = 64;  // variants in one set

// One compiled variant's parameters:
// "<id> <name> MWG NWG KWG MI WM WN SK VW LDS GM SG PREC PD".
struct FfDesc {
    int id = -1;
    std::string name;
    int mwg = 0, nwg = 0, kwg = 0, mi = 0, wm = 0, wn = 0, sk = 0, vw = 0, lds = 0, gm = 0, sg = 0;
    int prec = 0;  // 0 FP32 MFMA; 1 bf16x3, 2 bf16x6, 3 scaled fp16, 4 scaled fp16 in two pieces
                   // (16-bit MFMA, FP32 accumulation)
    int pd = 1;    // prefetch depth (compiled into the kernel; not a launch parameter)
    bool presplit() const { return prec > 0 && lds == 2; }
    int terms() const   // 16-bit pieces per value: bf16x3 2, bf16x6 3, fp16s 1, fp16x3 2
    {
        switch (prec) {
            case 1: case 4: return 2;
            case 2: return 3;
            default: return 1;
        }
    }
    bool scaled() const { return prec >= 3; }   // per-matrix power-of-two prescale
    int threads() const { return 64 * wm * wn * sk; }
};

// Read one descriptor from `is` and check its values; false if malformed.
bool ff_parse_descriptor(std::istream& is, FfDesc& d);

// A parsed set file: its form, target architecture, code-object directory
// (as written), members, and per training shape the winner and every
// member's log-slowdown (+inf where it failed), ntrain x k row-major.
struct FfSetFile {
    int form = 0;
    std::string arch, codedir;
    std::vector<FfDesc> members;
    std::vector<std::array<int64_t, 3>> shapes;
    std::vector<int> winners;
    std::vector<double> cost;
};

// Parse a set file.  Returns 0, or FF_ERR_IO / FF_ERR_PARSE with the reason
// in `err`.
int ff_read_set_file(const char* path, FfSetFile& out, std::string& err);

// Parse <dir>/manifest.txt.  Returns 0, or FF_ERR_IO / FF_ERR_PARSE.
int ff_read_manifest(const char* dir, std::vector<FfDesc>& out, std::string& err);
