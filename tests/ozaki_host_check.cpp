// CPU check of the residue arithmetic of the INT8-emulated FP64 products
// (paper_2408_04440_amd/csrc/ozaki_crt.h), run by tests/test_host_logic.py:
// reads integers P (sign and two 64-bit hex words) from stdin, forms their
// residues, recovers P with the library's CRT helpers and prints the bits of
// the double it rounds to; reads "m a p" lines for the residue conversions.
#include <cstdio>
#include <cstring>
#include <cmath>

#include "../paper_2408_04440_amd/csrc/ozaki_crt.h"

using namespace mpc;

int main()
{
    OzakiConst k;
    ozaki_const_init(&k);
    char kind[8];
    while (scanf("%7s", kind) == 1) {
        if (!strcmp(kind, "P")) {
            int neg;
            unsigned long long hi, lo;
            if (scanf("%d %llx %llx", &neg, &hi, &lo) != 3) return 2;
            unsigned __int128 mag = ((unsigned __int128)hi << 64) | lo;
            uint32_t S[4] = {0, 0, 0, 0};
            for (int l = 0; l < OZ_NMOD; ++l) {
                uint32_t r = (uint32_t)(mag % k.p[l]);
                if (neg && r) r = k.p[l] - r;  // residue of -mag
                crt_madd(S, r, k.W[l]);
                if (l % 3 == 2 || l == OZ_NMOD - 1) crt_reduce(S, k);
            }
            double v = crt_to_double(S, k);
            // the same residues through the three FP64 parts
            double sp[3] = {0.0, 0.0, 0.0};
            for (int l = 0; l < OZ_NMOD; ++l) {
                uint32_t r = (uint32_t)(mag % k.p[l]);
                if (neg && r) r = k.p[l] - r;
                crt_fma(sp, r, k.Wd[l]);
            }
            uint32_t S2[4];
            crt_parts_to_limbs(sp, k, S2);
            double v2 = crt_to_double(S2, k);
            unsigned long long bits, bits2;
            memcpy(&bits, &v, 8);
            memcpy(&bits2, &v2, 8);
            printf("%016llx %016llx\n", bits, bits2);
        } else if (!strcmp(kind, "sym")) {  // integer-valued double -> signed residue
            double a;
            unsigned p;
            if (scanf("%lf %u", &a, &p) != 2) return 2;
            printf("%d\n", (int)mod_sym(a, (double)p, 1.0 / (double)p));
        } else if (!strcmp(kind, "small")) {
            int x;
            unsigned p;
            if (scanf("%d %u", &x, &p) != 2) return 2;
            printf("%u\n", mod_small(x, p, 1.0f / (float)p));
        } else if (!strcmp(kind, "M")) {
            printf("%08x%08x%08x%08x\n", k.M[3], k.M[2], k.M[1], k.M[0]);
        } else {
            return 3;
        }
    }
    return 0;
}
