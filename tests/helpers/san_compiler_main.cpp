// Driver that runs the constraint compiler (ct_compile) in a standalone executable, so the test
// suite can build it with AddressSanitizer and UndefinedBehaviorSanitizer.  Test infrastructure
// only; the error reporter it provides stands in for the library's.
//
// Input file, text: a line "D", then per parameter a line "name r v_0 ... v_{r-1}", then a line
// "C", then C lines each holding one constraint.  Output file, text: the return code, the
// number of code words, the words, the C + 1 program offsets, then the error message.
#include <cstdint>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ct.h"

static std::string g_msg;
int ct_fail(int code, const std::string& msg) {
    g_msg = msg;
    return code;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    std::ifstream in(argv[1]);
    std::string line;
    std::getline(in, line);
    const int D = std::stoi(line);
    std::vector<std::string> names(D);
    std::vector<int64_t> values;
    std::vector<uint32_t> radices(D);
    for (int j = 0; j < D; ++j) {
        std::getline(in, line);
        std::istringstream ss(line);
        ss >> names[j] >> radices[j];
        for (uint32_t k = 0; k < radices[j]; ++k) {
            long long v;
            ss >> v;
            values.push_back(v);
        }
    }
    std::getline(in, line);
    const int C = std::stoi(line);
    std::vector<std::string> cons(C);
    for (int c = 0; c < C; ++c) std::getline(in, cons[c]);
    std::vector<const char*> np(D), cp(C > 0 ? C : 1);
    for (int j = 0; j < D; ++j) np[j] = names[j].c_str();
    for (int c = 0; c < C; ++c) cp[c] = cons[c].c_str();
    size_t chars = 0;
    for (const std::string& c : cons) chars += c.size();
    const uint32_t cap = (uint32_t)(64 + 64 * chars);
    std::vector<uint32_t> code(cap), offs(C + 1);
    uint32_t used = 0;
    const int rc = ct_compile(np.data(), (uint32_t)D, values.data(), radices.data(), cp.data(), (uint32_t)C,
                              code.data(), cap, offs.data(), &used);
    std::ofstream out(argv[2]);
    out << rc << "\n" << (rc == 0 ? used : 0) << "\n";
    for (uint32_t k = 0; rc == 0 && k < used; ++k) out << code[k] << " ";
    out << "\n";
    for (int c = 0; rc == 0 && c <= C; ++c) out << offs[c] << " ";
    out << "\n" << g_msg << "\n";
    return 0;
}
